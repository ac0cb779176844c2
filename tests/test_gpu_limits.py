"""Row pitch at the widest accepted image. The streaming kernels address a
workgroup's rows (at most 16 + 2 * 8 = 32 of them) through one buffer
descriptor of 2^30 bytes that starts at its first row, so the library accepts
W * (bytes per pixel) * 33 < 2^30 and rejects one column more with E_INVAL
before anything is launched. At the widest accepted FP32 width a band with
all 32 rows inside the image reads bytes up to 31 W * 4 + W * 4 - 1, just
under 2^30 (FP16/BF16: 31 W * 2 + W * 2 - 1 at their widest); q there must
match the FP64 oracle (sliding window, Eq. (2)) at the image's left and right
edges."""
import numpy as np
import pytest

from oracle import ref
from parity import check_maps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DESC_BYTES = 1 << 30
ROWS = 16 + 2 * 8 + 1
WINDOW, HALO = 17, 8


def widest(bpp: int) -> int:
    return (DESC_BYTES - 1) // (bpp * ROWS)


@pytest.mark.parametrize("dtype,bpp", [(torch.float32, 4), (torch.float16, 2)])
def test_one_column_past_the_bound_is_rejected(dtype, bpp):
    from paper_2509_21754_amd import Context, FitrigError

    W = widest(bpp) + 1
    assert W * bpp * ROWS >= DESC_BYTES and (W - 1) * bpp * ROWS < DESC_BYTES
    print(f"[limits] reject W={W} bpp={bpp}", flush=True)
    stack = torch.ones((3, 1, W), dtype=dtype, device="cuda")
    with Context(window=WINDOW, max_pixels=W, max_snap=3, branches=1) as ctx:
        with pytest.raises(FitrigError) as e:
            ctx.detect(stack, 6.0, as_dicts=False)
    assert e.value.code == -1


@pytest.mark.parametrize("dtype,bpp", [(torch.float32, 4), (torch.float16, 2), (torch.bfloat16, 2)])
def test_widest_image_matches_oracle_at_both_edges(dtype, bpp):
    """The oracle takes the stored values (FP16/BF16 widened exactly)."""
    from paper_2509_21754_amd import Context

    W, H = widest(bpp), 40
    print(f"[limits] accept {H}x{W} {dtype} window {WINDOW}", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(W)
    stack = (torch.randn((3, H, W), generator=g, device="cuda", dtype=torch.float32) + 3.0).to(dtype)
    qmap = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    with Context(window=WINDOW, max_pixels=H * W, max_snap=3, branches=1) as ctx:
        _, _, rc = ctx.detect(stack, 1e9, index_map=qmap, as_dicts=False)
    torch.cuda.synchronize()
    assert rc == 0
    for x0, x1 in ((0, 48), (W - 48, W)):
        xa, xb = max(0, x0 - HALO), min(W, x1 + HALO)
        X = stack[:, :, xa:xb].float().cpu().numpy()
        yy, xx = np.meshgrid(np.arange(H), np.arange(x0, x1), indexing="ij")
        cells = np.stack([np.zeros(yy.size, np.int64), yy.ravel(), (xx - xa).ravel()], 1)
        q_ref = ref.index_cells(X, cells, window=WINDOW).reshape(1, H, x1 - x0)
        check_maps(qmap[:, :, x0:x1].cpu().numpy(), q_ref, what=f"q[:, :, {x0}:{x1}]")


@pytest.mark.parametrize("dtype,bpp", [(torch.float32, 4), (torch.float16, 2)])
def test_widest_image_tile_mode_matches_oracle_at_both_edges(dtype, bpp):
    """Tile mode (Eq. (6), tile 32): each band of 32 rows is read through one
    descriptor; the tiles are independent, so the oracle runs on crops that
    start on a tile boundary. The last tile column is ragged."""
    from paper_2509_21754_amd import Context

    T, H = 32, 64
    W = widest(bpp)
    nt = -(-W // T)
    print(f"[limits] tile mode {H}x{W} {dtype}, {nt} tile columns (last {W - T * (nt - 1)} wide)", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(W + 1)
    stack = (torch.randn((3, H, W), generator=g, device="cuda", dtype=torch.float32) + 3.0).to(dtype)
    qmap = torch.empty((1, H // T, nt), dtype=torch.float32, device="cuda")
    with Context(mode=1, tile=T, max_pixels=H * W, max_snap=3, branches=1) as ctx:
        _, _, rc = ctx.detect(stack, 1e9, index_map=qmap, as_dicts=False)
    torch.cuda.synchronize()
    assert rc == 0
    for t0, t1 in ((0, 3), (nt - 3, nt)):
        X = stack[:, :, T * t0:min(W, T * t1)].float().cpu().numpy()
        q_ref = ref.index_maps(X, mode=ref.TILES, tile=T)
        check_maps(qmap[:, :, t0:t1].cpu().numpy(), q_ref, what=f"tiles {t0}:{t1}")
