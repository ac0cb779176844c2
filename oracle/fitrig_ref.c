/*
 * FITrig FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * GPU library is checked against. It is loaded only by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark. The product path
 * never links, loads or calls it, and it shares no code, header or constant
 * with the HIP library.
 *
 * Every step follows the paper (Li, Adamek & Armour, "FITrig", arXiv
 * 2509.21754) in its own order, in double precision, with no blocking,
 * fusion or reordering:
 *   - difference images D, the change image Delta = |D(s) - D(s+1)|, the
 *     reference substitute x_hat and the clamped ratio r: Sec. 2.2.4,
 *     Eqs. (2)-(5);
 *   - the index itself, 1 - mean(Delta) max(Delta) mean(r) / M^2, where
 *     M = max(max_s x, C): Eq. (2); the equivalent sum form used by the
 *     paper's kernel: Eq. (6), Sec. 2.3;
 *   - per-triple z-score and the selection {t : z_t > tau}: Sec. 2.4.1,
 *     Eqs. (8)-(9);
 *   - the image-frequency spectrum eta = h(|F[q(s) - mean q]|) and its
 *     z-score selection: Sec. 2.4.2, Eqs. (10)-(12).
 *
 * Readings where the paper is silent or ambiguous (each is listed in the
 * design notes of the repository):
 *   - the ratio uses |x_hat| unless r_signed is set (Eq. (4) literally
 *     divides by the signed value);
 *   - the reference frame of triple s (0-based) is frame s+1, the triple is
 *     frames s, s+1, s+2;
 *   - "per pixel" mode: an odd w x w window centred on each pixel, clipped
 *     at the image edge, mean = sum / (number of in-image pixels);
 *   - tile mode: non-overlapping tile x tile tiles in row-major order, the
 *     last row/column of tiles may be partial and uses its actual count;
 *   - the index map stores q = mean(Delta) max(Delta) mean(r), the part of
 *     Eq. (2) that varies between cells; tLISI = 1 - q / M^2. The z-score of
 *     Eq. (8) equals (q - mean q) / std q because tLISI is affine in q with
 *     a negative slope;
 *   - std uses the population normalisation (divide by the count);
 *   - MEDIAN_MAD: median (mean of the two middle values for an even count)
 *     and sigma = 1.482602218505602 * median |q - median|;
 *   - zero or non-finite spread gives no selection;
 *   - selection is strict (z > tau); candidates are 8-connected components,
 *     labelled by their lowest row-major index;
 *   - the transform over s is the unnormalised DFT of exact length n' with
 *     no padding, one-sided k = 1 .. floor(n'/2); h is the maximum
 *     magnitude (harm = 0) or the harmonic sum max_k sum_{j<=harm} A_{jk}
 *     with terms beyond floor(n'/2) dropped.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_SLIDING 0
#define REF_TILES 1
#define REF_MEAN_STD 0
#define REF_MEDIAN_MAD 1

/* One 8-connected component of selected cells. */
typedef struct {
  int64_t label;   /* lowest row-major index y*width + x of the component */
  int64_t n_pix;
  int64_t peak_y, peak_x;
  double peak_z, peak_q;
  double cy, cx;   /* z-weighted centroid */
  int64_t y0, x0, y1, x1;
} ref_comp;

static double load_px(const void* X, int in_f32, int64_t i) {
  if (in_f32) return (double)((const float*)X)[i];
  return ((const double*)X)[i];
}

/*
 * Per-pixel terms of triple s (frames s, s+1, s+2), Eqs. (3)-(5):
 *   D1 = |x(s+1) - x(s)|, D2 = |x(s+2) - x(s+1)|, Delta = |D1 - D2|,
 *   x_hat = x(s+1), or C where x(s+1) == 0,
 *   rho = Delta / |x_hat|  (Delta / x_hat when r_signed),
 *   r = rho if rho < 1 else 1.
 */
int ref_pixel_terms(const void* X, int in_f32, int n, int64_t H, int64_t W,
                    int s, int r_signed, double C, double* delta, double* r) {
  if (!X || n < 3 || s < 0 || s > n - 3 || H < 1 || W < 1) return -1;
  int64_t plane = H * W;
  for (int64_t p = 0; p < plane; ++p) {
    double x0 = load_px(X, in_f32, (int64_t)s * plane + p);
    double x1 = load_px(X, in_f32, (int64_t)(s + 1) * plane + p);
    double x2 = load_px(X, in_f32, (int64_t)(s + 2) * plane + p);
    double D1 = fabs(x1 - x0);
    double D2 = fabs(x2 - x1);
    double d = fabs(D1 - D2);
    double xh = (x1 == 0.0) ? C : x1;
    double rho = r_signed ? d / xh : d / fabs(xh);
    delta[p] = d;
    r[p] = (rho < 1.0) ? rho : 1.0;
  }
  return 0;
}

/* M = max(max over every frame and pixel, C): the normaliser of Eq. (2). */
double ref_normaliser(const void* X, int in_f32, int64_t count, double C) {
  double m = C;
  for (int64_t i = 0; i < count; ++i) {
    double v = load_px(X, in_f32, i);
    if (v > m) m = v;
  }
  return m;
}

/* mean(Delta) * max(Delta) * mean(r) over the rows [ya, yb) and columns
 * [xa, xb) of the precomputed Delta and r planes: the varying part of Eq. (2). */
static double region_q(const double* delta, const double* r, int64_t W,
                       int64_t ya, int64_t yb, int64_t xa, int64_t xb) {
  double sum_d = 0.0, max_d = -INFINITY, sum_r = 0.0;
  int64_t count = 0;
  for (int64_t y = ya; y < yb; ++y) {
    for (int64_t x = xa; x < xb; ++x) {
      double d = delta[y * W + x];
      sum_d += d;
      if (d > max_d) max_d = d;
      sum_r += r[y * W + x];
      ++count;
    }
  }
  return (sum_d / (double)count) * max_d * (sum_r / (double)count);
}

/*
 * q maps for every triple, q_out laid out [n-2][Ho][Wo]:
 *   sliding: Ho = H, Wo = W, window w (odd) centred on each pixel, clipped;
 *   tiles:   Ho = ceil(H / tile), Wo = ceil(W / tile), row-major tiles.
 */
int ref_index_maps(const void* X, int in_f32, int n, int64_t H, int64_t W,
                   int mode, int window, int tile, int r_signed, double C,
                   double* q_out) {
  if (!X || !q_out || n < 3 || H < 1 || W < 1) return -1;
  if (mode == REF_SLIDING && (window < 1 || window % 2 == 0)) return -1;
  if (mode == REF_TILES && tile < 1) return -1;
  if (mode != REF_SLIDING && mode != REF_TILES) return -1;
  int64_t plane = H * W;
  double* delta = (double*)malloc(sizeof(double) * plane);
  double* r = (double*)malloc(sizeof(double) * plane);
  if (!delta || !r) { free(delta); free(r); return -2; }
  int64_t Ho = (mode == REF_SLIDING) ? H : (H + tile - 1) / tile;
  int64_t Wo = (mode == REF_SLIDING) ? W : (W + tile - 1) / tile;
  int64_t half = (int64_t)(window / 2);
  for (int s = 0; s < n - 2; ++s) {
    ref_pixel_terms(X, in_f32, n, H, W, s, r_signed, C, delta, r);
    double* q = q_out + (int64_t)s * Ho * Wo;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t oy = 0; oy < Ho; ++oy) {
      for (int64_t ox = 0; ox < Wo; ++ox) {
        int64_t ya, yb, xa, xb;
        if (mode == REF_SLIDING) {
          ya = oy - half < 0 ? 0 : oy - half;
          yb = oy + half + 1 > H ? H : oy + half + 1;
          xa = ox - half < 0 ? 0 : ox - half;
          xb = ox + half + 1 > W ? W : ox + half + 1;
        } else {
          ya = oy * tile;
          yb = ya + tile > H ? H : ya + tile;
          xa = ox * tile;
          xb = xa + tile > W ? W : xa + tile;
        }
        q[oy * Wo + ox] = region_q(delta, r, W, ya, yb, xa, xb);
      }
    }
  }
  free(delta);
  free(r);
  return 0;
}

/*
 * Sliding-mode q at individual cells (s, y, x), for spot checks of inputs
 * too large for full maps. cells holds ncells triples (s, y, x).
 */
int ref_index_cells(const void* X, int in_f32, int n, int64_t H, int64_t W,
                    int window, int r_signed, double C, const int64_t* cells,
                    int64_t ncells, double* q_out) {
  if (!X || !cells || !q_out || n < 3 || window < 1 || window % 2 == 0) return -1;
  int64_t plane = H * W;
  int64_t half = window / 2;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < ncells; ++i) {
    int64_t s = cells[3 * i], y = cells[3 * i + 1], x = cells[3 * i + 2];
    double sum_d = 0.0, max_d = -INFINITY, sum_r = 0.0;
    int64_t count = 0;
    if (s < 0 || s > n - 3 || y < 0 || y >= H || x < 0 || x >= W) {
      q_out[i] = NAN;
      continue;
    }
    for (int64_t yy = y - half; yy <= y + half; ++yy) {
      if (yy < 0 || yy >= H) continue;
      for (int64_t xx = x - half; xx <= x + half; ++xx) {
        if (xx < 0 || xx >= W) continue;
        int64_t p = yy * W + xx;
        double x0 = load_px(X, in_f32, s * plane + p);
        double x1 = load_px(X, in_f32, (s + 1) * plane + p);
        double x2 = load_px(X, in_f32, (s + 2) * plane + p);
        double D1 = fabs(x1 - x0), D2 = fabs(x2 - x1);
        double d = fabs(D1 - D2);
        double xh = (x1 == 0.0) ? C : x1;
        double rho = r_signed ? d / xh : d / fabs(xh);
        double rr = (rho < 1.0) ? rho : 1.0;
        sum_d += d;
        if (d > max_d) max_d = d;
        sum_r += rr;
        ++count;
      }
    }
    q_out[i] = (sum_d / (double)count) * max_d * (sum_r / (double)count);
  }
  return 0;
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* Median of v[0..n) (sorts v in place). */
static double median_inplace(double* v, int64_t n) {
  qsort(v, (size_t)n, sizeof(double), cmp_double);
  if (n % 2 == 1) return v[n / 2];
  return 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

/*
 * Spread of one map, Sec. 2.4.1 Eq. (8) (mean and standard deviation of the
 * map), or the robust median / MAD variant.
 */
int ref_spread(const double* q, int64_t count, int estimator, double* mu,
               double* sigma) {
  if (!q || count < 1 || !mu || !sigma) return -1;
  if (estimator == REF_MEAN_STD) {
    double s = 0.0;
    for (int64_t i = 0; i < count; ++i) s += q[i];
    double m = s / (double)count;
    double v = 0.0;
    for (int64_t i = 0; i < count; ++i) v += (q[i] - m) * (q[i] - m);
    *mu = m;
    *sigma = sqrt(v / (double)count);
    return 0;
  }
  if (estimator == REF_MEDIAN_MAD) {
    double* tmp = (double*)malloc(sizeof(double) * count);
    if (!tmp) return -2;
    memcpy(tmp, q, sizeof(double) * count);
    double med = median_inplace(tmp, count);
    for (int64_t i = 0; i < count; ++i) tmp[i] = fabs(q[i] - med);
    double mad = median_inplace(tmp, count);
    free(tmp);
    *mu = med;
    *sigma = 1.482602218505602 * mad;
    return 0;
  }
  return -1;
}

/*
 * Selection {c : (q_c - mu) / sigma > tau} (Eqs. (8)-(9), (11)-(12)) and its
 * 8-connected components, found by a flood fill started from each
 * unlabelled selected cell in row-major order (so the starting cell is the
 * lowest index of its component). Components are written in label order.
 * Returns the number of components (all of them are counted; at most cap
 * are written), or -1 on bad arguments. sel (nullable) receives the mask.
 */
int64_t ref_components(const double* q, int64_t Ho, int64_t Wo, double mu,
                       double sigma, double tau, uint8_t* sel_out,
                       ref_comp* out, int64_t cap) {
  if (!q || Ho < 1 || Wo < 1) return -1;
  int64_t N = Ho * Wo;
  uint8_t* sel = (uint8_t*)calloc((size_t)N, 1);
  uint8_t* seen = (uint8_t*)calloc((size_t)N, 1);
  int64_t* stack = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  if (!sel || !seen || !stack) { free(sel); free(seen); free(stack); return -2; }
  int ok = (sigma > 0.0) && isfinite(sigma) && isfinite(mu);
  if (ok)
    for (int64_t i = 0; i < N; ++i) sel[i] = ((q[i] - mu) / sigma > tau) ? 1 : 0;
  if (sel_out) memcpy(sel_out, sel, (size_t)N);
  int64_t ncomp = 0;
  for (int64_t start = 0; start < N; ++start) {
    if (!sel[start] || seen[start]) continue;
    ref_comp c;
    c.label = start;
    c.n_pix = 0;
    c.peak_y = c.peak_x = -1;
    c.peak_z = -INFINITY;
    c.peak_q = 0.0;
    c.y0 = c.x0 = INT64_MAX;
    c.y1 = c.x1 = INT64_MIN;
    double sw = 0.0, swy = 0.0, swx = 0.0;
    int64_t best_idx = -1;
    int64_t top = 0;
    stack[top++] = start;
    seen[start] = 1;
    while (top > 0) {
      int64_t idx = stack[--top];
      int64_t y = idx / Wo, x = idx % Wo;
      double z = (q[idx] - mu) / sigma;
      c.n_pix += 1;
      if (z > c.peak_z || (z == c.peak_z && idx < best_idx)) {
        c.peak_z = z;
        c.peak_q = q[idx];
        best_idx = idx;
      }
      sw += z;
      swy += z * (double)y;
      swx += z * (double)x;
      if (y < c.y0) c.y0 = y;
      if (y > c.y1) c.y1 = y;
      if (x < c.x0) c.x0 = x;
      if (x > c.x1) c.x1 = x;
      for (int dy = -1; dy <= 1; ++dy) {
        for (int dx = -1; dx <= 1; ++dx) {
          if (dy == 0 && dx == 0) continue;
          int64_t yy = y + dy, xx = x + dx;
          if (yy < 0 || yy >= Ho || xx < 0 || xx >= Wo) continue;
          int64_t j = yy * Wo + xx;
          if (sel[j] && !seen[j]) {
            seen[j] = 1;
            stack[top++] = j;
          }
        }
      }
    }
    c.peak_y = best_idx / Wo;
    c.peak_x = best_idx % Wo;
    c.cy = swy / sw;
    c.cx = swx / sw;
    if (out && ncomp < cap) out[ncomp] = c;
    ++ncomp;
  }
  free(sel);
  free(seen);
  free(stack);
  return ncomp;
}

/*
 * Image-frequency spectrum, Sec. 2.4.2 Eq. (10). cube is laid out
 * [nprime][ntiles] (time-major). For each tile: v = q(s) - mean_s q,
 * X_k = sum_s v_s exp(-2 pi i k s / nprime), A_k = |X_k| for
 * k = 1 .. floor(nprime/2); eta = max_k A_k (harm == 0) or
 * max_k sum_{j=1..harm, j k <= floor(nprime/2)} A_{jk} (harm >= 2).
 */
int ref_eta(const double* cube, int nprime, int64_t ntiles, int harm,
            double* eta) {
  if (!cube || !eta || nprime < 2 || ntiles < 1 || harm < 0 || harm == 1) return -1;
  int K = nprime / 2;
  double* v = (double*)malloc(sizeof(double) * nprime);
  double* A = (double*)malloc(sizeof(double) * (K + 1));
  if (!v || !A) { free(v); free(A); return -2; }
  const double two_pi = 6.283185307179586476925286766559;
  for (int64_t t = 0; t < ntiles; ++t) {
    double mean = 0.0;
    for (int s = 0; s < nprime; ++s) mean += cube[(int64_t)s * ntiles + t];
    mean /= (double)nprime;
    for (int s = 0; s < nprime; ++s) v[s] = cube[(int64_t)s * ntiles + t] - mean;
    A[0] = 0.0;
    for (int k = 1; k <= K; ++k) {
      double re = 0.0, im = 0.0;
      for (int s = 0; s < nprime; ++s) {
        /* exact reduction of the phase k*s/nprime before the cos/sin */
        double ang = two_pi * (double)(((int64_t)k * s) % nprime) / (double)nprime;
        re += v[s] * cos(ang);
        im -= v[s] * sin(ang);
      }
      A[k] = sqrt(re * re + im * im);
    }
    double best = 0.0;
    for (int k = 1; k <= K; ++k) {
      double val = 0.0;
      if (harm == 0) {
        val = A[k];
      } else {
        for (int j = 1; j <= harm && (int64_t)j * k <= K; ++j) val += A[j * k];
      }
      if (k == 1 || val > best) best = val;
    }
    eta[t] = (K >= 1) ? best : 0.0;
  }
  free(v);
  free(A);
  return 0;
}

int ref_abi_version(void) { return 1; }

/* Threads of the OpenMP loops (for timing the oracle at a given core count;
 * the arithmetic does not depend on it). */
void ref_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int ref_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
