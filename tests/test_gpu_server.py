"""GPU tests of the serving form through the C ABI: every result of a mix of
fields served concurrently equals the same frames (the field's two carried
snapshots followed by the request's) run alone through fitrig_detect, and
matches the FP64 oracle; requests of a field run in order; admission by
memory."""
import numpy as np
import pytest

from oracle import ref
from parity import check_candidates, structured_stack

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def _alone(frames_t, tau, **cfg):
    from paper_2509_21754_amd import Context

    with Context(**cfg) as ctx:
        cands, stats, rc = ctx.detect(frames_t, tau, as_dicts=False)
    return cands, stats, rc


def _plan(seed):
    """Fields (H, W, dtype) and an interleaved list of (field, n_new)."""
    rng = np.random.default_rng(seed)
    fields = {0: (70, 300, "f32"), 1: (33, 530, "f16"), 2: (64, 256, "f32"), 3: (5, 7, "bf16"),
              4: (128, 260, "f32")}
    reqs = []
    left = {f: 4 for f in fields}
    first = {f: True for f in fields}
    while any(left.values()):
        f = int(rng.choice([k for k, v in left.items() if v]))
        n = int(rng.integers(3, 7)) if first[f] else int(rng.integers(1, 6))
        first[f] = False
        left[f] -= 1
        reqs.append((f, n))
    return fields, reqs


@pytest.mark.parametrize("branches,extra,graphs", [(1, {}, 1), (3, {}, 1), (3, {}, 0), (3, dict(sigma_est=1), 1),
                                                   (3, dict(mode=1, tile=8), 1)])
def test_server_mix_equals_alone(branches, extra, graphs):
    from paper_2509_21754_amd import Server

    tau = 4.0
    cfg = dict(window=5, branches=branches, tile=16)
    cfg.update(extra)
    fields, reqs = _plan(7 + branches)
    frames = {f: [] for f in fields}   # every frame submitted so far, host float copies
    submitted = []
    keep = []
    with Server(n_slots=3, max_fields=8, graphs=graphs, **cfg) as srv:
        for i, (f, n) in enumerate(reqs):
            H, W, dt = fields[f]
            X = structured_stack(100 * f + i, n, H, W)
            t = torch.from_numpy(X).to(DT[dt]).cuda()
            torch.cuda.synchronize()
            keep.append(t)
            prev = frames[f][-2:]
            used = t.float().cpu().numpy()
            frames[f].extend(list(used))
            tk = srv.submit(f, t, tau)
            submitted.append((tk, f, len(frames[f]) - n - len(prev), np.stack(prev + list(used)), dt))
        results = [srv.poll(tk, as_dicts=False) for tk, *_ in submitted]
        done = {tk: r for (tk, *_), r in zip(submitted, results)}
        for (tk, f, first, used, dt), r in zip(submitted, results):
            assert r["status"] in (0, -4), r["status"]
            assert r["replayed"] == graphs
            assert r["field_id"] == f
            assert r["first_triple"] == first
            assert r["n_triples"] == used.shape[0] - 2
            frames_t = torch.from_numpy(used).to(DT[dt]).cuda()
            alone, stats, rc = _alone(frames_t, tau, **cfg)
            got = r["cands"].copy()
            img = got["branch"] == ref.IMAGE
            got["triple"][img] -= first
            assert got.tobytes() == alone.tobytes(), (tk, f)
            # the running M covers every frame of the field so far and C
            seen = np.stack(frames[f][:first + used.shape[0]])
            assert r["M"] == max(float(seen.max()), 1e-6)
            out = ref.detect(used.astype(np.float64), tau=tau, window=5, branches=branches, tile=cfg["tile"],
                             sigma_est=cfg.get("sigma_est", 0), mode=cfg.get("mode", 0))
            from paper_2509_21754_amd.fitrig import _rec_dict
            check_candidates([_rec_dict(x) for x in alone], out, tau)
        # per-field submission order
        for f in fields:
            mine = [done[tk] for tk, ff, *_ in submitted if ff == f]
            for a, b in zip(mine, mine[1:]):
                assert b["t_start_ns"] >= a["t_done_ns"]
                assert b["first_triple"] == a["first_triple"] + a["n_triples"]
        for tk, *_ in submitted:
            srv.release(tk)


def test_server_graph_replays_of_one_shape():
    """One slot serves one field with requests of one shape: the captured
    launch sequence is replayed again and again (torch work and host
    synchronisations between the replays), and every result equals the same
    frames run alone."""
    from paper_2509_21754_amd import Server

    tau = 4.0
    cfg = dict(window=7, branches=3, tile=16)
    prev = None
    with Server(n_slots=1, graphs=1, **cfg) as srv:
        for i in range(6):
            X = structured_stack(300 + i, 5, 96, 300)
            t = torch.from_numpy(X).cuda()
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between the replays
            torch.cuda.synchronize()
            tk = srv.submit(0, t, tau)
            r = srv.poll(tk, as_dicts=False)
            float(junk)
            assert r["status"] in (0, -4) and r["replayed"] == 1
            used = X if prev is None else np.concatenate([prev, X])
            alone, _, _ = _alone(torch.from_numpy(np.ascontiguousarray(used)).cuda(), tau, **cfg)
            got = r["cands"].copy()
            img = got["branch"] == ref.IMAGE
            got["triple"][img] -= r["first_triple"]
            assert got.tobytes() == alone.tobytes(), i
            prev = X[-2:]
            srv.release(tk)


def test_server_presized_slots_bound_device_memory():
    """With capacity hints every slot is sized at create and charged against
    the budget; the device memory the server takes stays within the budget,
    also when a request larger than the hints grows a slot."""
    from paper_2509_21754_amd import FitrigError, Server

    stacks = [torch.from_numpy(structured_stack(400 + i, 6, 256, 512)).cuda() for i in range(8)]
    big = torch.zeros((6, 600, 600), device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    budget = 1 << 30
    with pytest.raises(FitrigError):
        Server(n_slots=4, mem_budget=1 << 20, max_pixels=256 * 512, max_snap=6, window=7)
    with Server(n_slots=4, mem_budget=budget, max_pixels=256 * 512, max_snap=6, window=7) as srv:
        low = free0 - torch.cuda.mem_get_info()[0]
        tks = [srv.submit(i % 3, s, 5.0) for i, s in enumerate(stacks)]
        tks.append(srv.submit(99, big, 5.0))    # more pixels than the hints
        for tk in tks:
            r = srv.poll(tk)
            assert r["status"] in (0, -4)
            low = max(low, free0 - torch.cuda.mem_get_info()[0])
            srv.release(tk)
    # slack for the runtime's own per-stream and per-graph memory
    assert low <= budget + (64 << 20), low


def test_server_admission_by_memory():
    from paper_2509_21754_amd import FitrigError, Server

    X = torch.from_numpy(structured_stack(5, 4, 40, 300)).cuda()
    with Server(n_slots=2, mem_budget=1024, window=5) as srv:
        assert srv.submit(0, X, 5.0, blocking=False) is None
        with pytest.raises(FitrigError):
            srv.submit(0, X, 5.0, blocking=True)     # alone larger than the budget
    with Server(n_slots=2, window=5) as srv:
        tk = srv.submit(0, X, 5.0)
        r = srv.poll(tk)
        assert r["status"] == 0
        srv.release(tk)
        with pytest.raises(FitrigError):
            srv.poll(tk)
        with pytest.raises(FitrigError):
            srv.submit(1, X[:2].contiguous(), 5.0)    # a field's first request needs three frames
        tk2 = srv.submit(0, X[:1].contiguous(), 5.0)  # later requests may bring a single frame
        r2 = srv.poll(tk2)
        assert r2["n_triples"] == 1 and r2["first_triple"] == 2


def test_server_evicts_least_recently_used_idle_field():
    from paper_2509_21754_amd import Server

    X = torch.from_numpy(structured_stack(9, 5, 40, 300)).cuda()
    one = X[:1].contiguous()
    with Server(n_slots=2, max_fields=2, window=5) as srv:
        for f in (0, 1):
            srv.poll(srv.submit(f, X, 5.0))
        srv.poll(srv.submit(1, one, 5.0))          # field 1 used last
        r2 = srv.poll(srv.submit(2, X, 5.0))       # evicts field 0
        assert r2["first_triple"] == 0
        r1 = srv.poll(srv.submit(1, one, 5.0))     # field 1 kept its frames
        assert r1["first_triple"] == 4 and r1["n_triples"] == 1
        r0 = srv.poll(srv.submit(0, X, 5.0))       # field 0 starts over (evicts field 2)
        assert r0["first_triple"] == 0 and r0["n_triples"] == 3


@pytest.mark.parametrize("branches,tile", [(2, 16), (3, 32)])
def test_server_freq_window_covers_field_history(branches, tile):
    """With freq_window > 0 a request's frequency branch transforms the field's
    last freq_window triples (tile cube kept per field): its candidates equal
    those of the frames covering that window run alone."""
    from paper_2509_21754_amd import Server
    from paper_2509_21754_amd.fitrig import _rec_dict

    tau, win = 2.5, 6
    cfg = dict(window=5, branches=branches, tile=tile)
    H, W = 96, 200
    frames = []
    n_freq = 0
    with Server(n_slots=2, freq_window=win, **cfg) as srv:
        for i, n in enumerate([3, 2, 1, 4, 3, 1]):
            X = structured_stack(300 + i, n, H, W)
            t = torch.from_numpy(X).cuda()
            torch.cuda.synchronize()
            frames.extend(list(X))
            tk = srv.submit(0, t, tau)
            r = srv.poll(tk, as_dicts=False)
            assert r["status"] == 0
            T = len(frames) - 2
            nf = min(T, win)
            assert r["freq_triples"] == (nf if nf >= 4 else 0)
            got = r["cands"]
            gf = got[got["branch"] == ref.FREQ]
            if nf < 4:
                assert len(gf) == 0
            else:
                used = np.stack(frames[T - nf:T + 2])
                alone, _, rc = _alone(torch.from_numpy(used).cuda(), tau, **cfg)
                assert rc == 0
                af = alone[alone["branch"] == ref.FREQ]
                assert gf.tobytes() == af.tobytes(), i
                n_freq += len(af)
                out = ref.detect(used.astype(np.float64), tau=tau, window=5, branches=branches, tile=tile)
                check_candidates([_rec_dict(x) for x in alone], out, tau)
            srv.release(tk)
    assert n_freq > 0


@pytest.mark.parametrize("branches,extra,graphs", [(5, {}, 1), (7, {}, 0), (5, dict(sigma_est=1), 1)])
def test_server_freq_window_pixel_history(branches, extra, graphs):
    """With freq_window > 0 the per-pixel frequency branch of a request runs
    over the field's last freq_window index maps (kept per field in a ring,
    across requests of any size): its candidates equal those of the frames
    covering that window run alone, and match the oracle. Two fields, one of
    them with a ragged plane, are interleaved so that each keeps its own ring."""
    from paper_2509_21754_amd import Server
    from paper_2509_21754_amd.fitrig import _rec_dict

    tau, win = 2.5, 6
    cfg = dict(window=5, branches=branches, tile=16)
    cfg.update(extra)
    shapes = {0: (96, 200), 1: (37, 203)}
    sizes = {0: [3, 2, 1, 4, 3, 1, 5], 1: [4, 1, 1, 7, 2]}
    order = [0, 1, 0, 0, 1, 0, 1, 0, 1, 0, 1, 0]
    frames = {0: [], 1: []}
    nxt = {0: 0, 1: 0}
    n_px = 0
    with Server(n_slots=2, freq_window=win, graphs=graphs, **cfg) as srv:
        for i, f in enumerate(order):
            n = sizes[f][nxt[f]]
            nxt[f] += 1
            H, W = shapes[f]
            X = structured_stack(500 + 17 * f + i, n, H, W)
            t = torch.from_numpy(X).cuda()
            torch.cuda.synchronize()
            frames[f].extend(list(X))
            tk = srv.submit(f, t, tau)
            r = srv.poll(tk, as_dicts=False)
            assert r["status"] == 0, (i, f)
            T = len(frames[f]) - 2
            nf = min(T, win)
            got = r["cands"]
            gp = got[got["branch"] == ref.FREQ_PIXEL]
            if nf < 4:
                assert len(gp) == 0
            else:
                used = np.stack(frames[f][T - nf:T + 2])
                alone, _, rc = _alone(torch.from_numpy(used).cuda(), tau, **cfg)
                assert rc == 0
                ap = alone[alone["branch"] == ref.FREQ_PIXEL]
                assert gp.tobytes() == ap.tobytes(), (i, f, T)
                n_px += len(ap)
                out = ref.detect(used.astype(np.float64), tau=tau, window=5, branches=ref.FREQ_PIXEL, tile=16,
                                 sigma_est=cfg.get("sigma_est", 0))
                check_candidates([_rec_dict(x) for x in ap], out, tau)
            srv.release(tk)
    assert nxt == {0: len(sizes[0]), 1: len(sizes[1])}
    assert n_px > 0
