// D-SSIM term of the photometric energy (Sec. 3.4, eq. 8) on gfx950: per view, the loss
// 1 - mean SSIM over its three channels and pixels, and its gradient with respect to the
// rendered colour.  SSIM(p) = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)
// (s_x^2 + s_y^2 + C2)) over an 11 x 11 Gaussian window (standard deviation 1.5, weights
// summing to 1), pixels outside the image counting as 0, s^2 = E[x^2] - mu^2.
//
// Two stencil passes, each a 32 x 32 output tile per workgroup with its 5-pixel halo staged in
// LDS and the window applied as two 11-tap passes (the Gaussian window is separable).  Both
// passes are register-blocked: in the horizontal pass a thread reads 14 staged values of a row
// (four 16-byte LDS reads) and produces 4 adjacent columns; in the vertical pass it reads 14
// rows of one column and produces 4 adjacent rows.  Every output sums its 11 taps in the same
// order as a one-output-per-thread loop would.
//   k_ssim_stats: the five local moments -> SSIM(p) (summed per workgroup) and the three maps
//     A = dS/dmu_x - 2 mu_x B - mu_y C, B = dS/ds_xx, C = dS/ds_xy;
//   k_ssim_grad / k_photo_seeds: dL/dx(p) = -(1/N) (W*A + 2 x(p) W*B + y(p) W*C)(p), W* the
//     same window sum (the window is symmetric), N = 3 W H of the view;
// then k_ssim_loss adds the workgroups' sums of each view.
#include "tsr_device.h"
#include "tsr_internal.h"

#include <math.h>
#include <string.h>

namespace tsr {

constexpr float kSsimC1 = 0.01f * 0.01f;
constexpr float kSsimC2 = 0.03f * 0.03f;
constexpr int kSsimTaps = 2 * kSsimR + 1;
constexpr int kSsimIW = kSsimTW + 2 * kSsimR;   // staged columns
constexpr int kSsimIH = kSsimTH + 2 * kSsimR;   // staged rows
constexpr int kSsimLW = 44;                     // LDS row stride of the staged values (16-byte rows)
constexpr int kSsimBlk = 4;                     // outputs per thread in each pass
constexpr int kSsimSpan = kSsimBlk + 2 * kSsimR;   // inputs a thread reads per pass (14)
static_assert(kSsimTW == 32 && kSsimTH == 32, "a 256-thread workgroup: 32 columns x 8 groups of 4 rows");
static_assert(kSsimLW % 4 == 0 && kSsimLW >= kSsimIW && (kSsimTW - kSsimBlk) + 16 <= kSsimLW,
              "the horizontal pass reads four aligned float4 per row inside the staged row");

struct SsimTile {
  int v, ch, x0, y0, W, H;
  int64_t plane;          // offset of this channel plane in the packed colour arrays
};

// Workgroups are dealt round-robin to the 8 XCDs: each XCD gets a contiguous range of tiles
// (grid padded to a multiple of 8), so the halo a tile shares with the tiles above and below
// it is read through the same L2.  Returns the tile (channel-major over the views) or -1.
__device__ __forceinline__ int ssim_block(const SsimTable& t) {
  const int total = t.blk_off[t.n_views];
  const int per = (total + 7) >> 3;
  const int idx = (int)(blockIdx.x >> 3);
  const int b = (int)(blockIdx.x & 7) * per + idx;
  return (idx < per && b < total) ? b : -1;
}

static unsigned ssim_grid(const SsimTable& t) { return 8u * (unsigned)((t.blk_off[t.n_views] + 7) / 8); }

__device__ __forceinline__ SsimTile ssim_tile(const SsimTable& t, int b) {
  SsimTile s;
  int v = 0;
  for (int i = 1; i < t.n_views; ++i)
    if (b >= t.blk_off[i]) v = i;
  const int local = b - t.blk_off[v];
  const int ntile = t.tiles_x[v] * t.tiles_y[v];
  s.v = v;
  s.ch = local / ntile;
  const int tile = local - s.ch * ntile;
  s.x0 = (tile % t.tiles_x[v]) * kSsimTW;
  s.y0 = (tile / t.tiles_x[v]) * kSsimTH;
  s.W = t.width[v];
  s.H = t.height[v];
  s.plane = 3 * t.pix_off[v] + (int64_t)s.ch * s.W * s.H;
  return s;
}

// Stages the tile's window of Q images (zero outside the image) into in[q][row][col]: every
// load of the thread is issued before the first LDS store, so their latencies overlap.  Entry
// i = tid + 256 k sits at row i / 42, column i % 42; from one entry to the thread's next the
// row advances by 6 and the column by 4 (256 = 6 * 42 + 4), so no division is repeated, and a
// window wholly inside the image (most tiles) skips the per-entry bounds tests.
constexpr int kSsimStageIters = (kSsimIH * kSsimIW + 255) / 256;
static_assert(kSsimIW == 42 && 256 == 6 * kSsimIW + 4, "staging steps of 6 rows and 4 columns");

template <int Q>
__device__ __forceinline__ void ssim_stage(const SsimTile& s, const float* const* src, float (*in)[kSsimIH][kSsimLW]) {
  const int x0 = s.x0 - kSsimR, y0 = s.y0 - kSsimR;
  const bool interior = x0 >= 0 && y0 >= 0 && x0 + kSsimIW <= s.W && y0 + kSsimIH <= s.H;   // workgroup-uniform
  const float* base[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) base[q] = src[q] + s.plane;
  int r = (int)threadIdx.x / kSsimIW, c = (int)threadIdx.x - r * kSsimIW;
  float v[kSsimStageIters][Q];
  int rr[kSsimStageIters], cc[kSsimStageIters];
#pragma unroll
  for (int it = 0; it < kSsimStageIters; ++it) {
    const int gx = x0 + c, gy = y0 + r;
    const bool ld = r < kSsimIH && (interior || (gx >= 0 && gx < s.W && gy >= 0 && gy < s.H));
    const int off = gy * s.W + gx;         // < 2^28 for images up to 16384 x 16384
#pragma unroll
    for (int q = 0; q < Q; ++q) v[it][q] = ld ? base[q][off] : 0.f;
    rr[it] = r;
    cc[it] = c;
    c += 4;
    r += 6;
    if (c >= kSsimIW) {
      c -= kSsimIW;
      ++r;
    }
  }
#pragma unroll
  for (int it = 0; it < kSsimStageIters; ++it) {
    if (rr[it] < kSsimIH) {
#pragma unroll
      for (int q = 0; q < Q; ++q) in[q][rr[it]][cc[it]] = v[it][q];
    }
  }
}

// The kSsimSpan staged values of row r from column c0 (a multiple of 4) in four 16-byte reads.
__device__ __forceinline__ void ssim_row_span(const float* row, int c0, float v[16]) {
  const float4* p = reinterpret_cast<const float4*>(row + c0);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float4 a = p[j];
    v[4 * j] = a.x; v[4 * j + 1] = a.y; v[4 * j + 2] = a.z; v[4 * j + 3] = a.w;
  }
}

// Horizontal 11-tap pass of Q staged images into hs[q][row][col] (rows of the whole staged
// height, the tile's columns), 4 adjacent columns per task.
template <int Q>
__device__ __forceinline__ void ssim_hpass(const float* g, float (*in)[kSsimIH][kSsimLW],
                                           float (*hs)[kSsimIH][kSsimTW]) {
  constexpr int kGroups = kSsimTW / kSsimBlk;
  for (int task = threadIdx.x; task < kSsimIH * kGroups; task += blockDim.x) {
    const int r = task / kGroups, c0 = (task - r * kGroups) * kSsimBlk;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      float v[16];
      ssim_row_span(&in[q][r][0], c0, v);
#pragma unroll
      for (int o = 0; o < kSsimBlk; ++o) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kSsimTaps; ++k) acc = fmaf(g[k], v[o + k], acc);
        hs[q][r][c0 + o] = acc;
      }
    }
  }
}

// Vertical 11-tap pass of Q horizontal sums at column c for rows r0 .. r0 + 3 of the tile.
template <int Q>
__device__ __forceinline__ void ssim_vpass(const float* g, float (*hs)[kSsimIH][kSsimTW], int r0, int c,
                                           float m[kSsimBlk][Q]) {
#pragma unroll
  for (int o = 0; o < kSsimBlk; ++o)
#pragma unroll
    for (int q = 0; q < Q; ++q) m[o][q] = 0.f;
#pragma unroll
  for (int k = 0; k < kSsimSpan; ++k) {
    float v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = hs[q][r0 + k][c];
#pragma unroll
    for (int o = 0; o < kSsimBlk; ++o) {
      const int kk = k - o;              // tap of output row r0 + o
      if (kk >= 0 && kk < kSsimTaps) {
#pragma unroll
        for (int q = 0; q < Q; ++q) m[o][q] = fmaf(g[kk], v[q], m[o][q]);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_ssim_stats(const float* __restrict__ color, const float* __restrict__ target,
                                                    SsimTable t, float* __restrict__ abc, int64_t n3,
                                                    double* __restrict__ partial) {
  __shared__ __align__(16) float in[2][kSsimIH][kSsimLW];
  __shared__ float hs[5][kSsimIH][kSsimTW];
  __shared__ double red[4];
  const int b = ssim_block(t);
  if (b < 0) return;                       // whole workgroup
  const SsimTile s = ssim_tile(t, b);
  const float* src[2] = {color, target};
  ssim_stage<2>(s, src, in);
  __syncthreads();
  // horizontal pass of x, y, x^2, y^2, x y: the squares and product formed once per staged value
  constexpr int kGroups = kSsimTW / kSsimBlk;
  for (int task = threadIdx.x; task < kSsimIH * kGroups; task += blockDim.x) {
    const int r = task / kGroups, c0 = (task - r * kGroups) * kSsimBlk;
    float x[16], y[16];
    ssim_row_span(&in[0][r][0], c0, x);
    ssim_row_span(&in[1][r][0], c0, y);
    float xx[kSsimSpan], yy[kSsimSpan], xy[kSsimSpan];
#pragma unroll
    for (int k = 0; k < kSsimSpan; ++k) {
      xx[k] = x[k] * x[k];
      yy[k] = y[k] * y[k];
      xy[k] = x[k] * y[k];
    }
#pragma unroll
    for (int o = 0; o < kSsimBlk; ++o) {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
      for (int k = 0; k < kSsimTaps; ++k) {
        const float w = t.g[k];
        a0 = fmaf(w, x[o + k], a0);
        a1 = fmaf(w, y[o + k], a1);
        a2 = fmaf(w, xx[o + k], a2);
        a3 = fmaf(w, yy[o + k], a3);
        a4 = fmaf(w, xy[o + k], a4);
      }
      hs[0][r][c0 + o] = a0; hs[1][r][c0 + o] = a1; hs[2][r][c0 + o] = a2; hs[3][r][c0 + o] = a3; hs[4][r][c0 + o] = a4;
    }
  }
  __syncthreads();
  // vertical pass and the per-pixel SSIM terms, rows r0 .. r0 + 3 of column c
  const int c = threadIdx.x & (kSsimTW - 1), r0 = (threadIdx.x / kSsimTW) * kSsimBlk;
  float m[kSsimBlk][5];
  ssim_vpass<5>(t.g, hs, r0, c, m);
  double sum = 0.0;
  const int gx = s.x0 + c;
#pragma unroll
  for (int o = 0; o < kSsimBlk; ++o) {
    const int gy = s.y0 + r0 + o;
    if (gx >= s.W || gy >= s.H) continue;
    const float mx = m[o][0], my = m[o][1];
    const float sxx = m[o][2] - mx * mx, syy = m[o][3] - my * my, sxy = m[o][4] - mx * my;
    const float n1 = 2.f * mx * my + kSsimC1, n2 = 2.f * sxy + kSsimC2;
    const float d1 = mx * mx + my * my + kSsimC1, d2 = sxx + syy + kSsimC2;
    // one division: 1/d1 = d2 inv and 1/d2 = d1 inv
    const float inv = 1.f / (d1 * d2);
    const float S = n1 * n2 * inv;
    const float B = -S * d1 * inv;
    const float C = 2.f * n1 * inv;
    const float A = 2.f * my * n2 * inv - 2.f * mx * S * d2 * inv - 2.f * mx * B - my * C;
    const int64_t e = s.plane + (int64_t)gy * s.W + gx;
    abc[e] = A;
    abc[n3 + e] = B;
    abc[2 * n3 + e] = C;
    sum += (double)S;
  }
  // workgroup sum of SSIM -> partial[blockIdx.x]
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) partial[b] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_ssim_grad(const float* __restrict__ color, const float* __restrict__ target,
                                                   SsimTable t, const float* __restrict__ abc, int64_t n3, float weight,
                                                   int accumulate, float* __restrict__ grad) {
  __shared__ __align__(16) float in[3][kSsimIH][kSsimLW];
  __shared__ float hs[3][kSsimIH][kSsimTW];
  const int b = ssim_block(t);
  if (b < 0) return;                       // whole workgroup
  const SsimTile s = ssim_tile(t, b);
  // this thread's outputs: rows r0 .. r0 + 3 of column c; their colour values are loaded first
  const int c = threadIdx.x & (kSsimTW - 1), r0 = (threadIdx.x / kSsimTW) * kSsimBlk;
  const int gx = s.x0 + c;
  float xo[kSsimBlk], yo[kSsimBlk], go[kSsimBlk];
#pragma unroll
  for (int o = 0; o < kSsimBlk; ++o) {
    const int gy = s.y0 + r0 + o;
    const bool ok = gx < s.W && gy < s.H;
    const int64_t e = s.plane + (int64_t)gy * s.W + gx;
    xo[o] = ok ? color[e] : 0.f;
    yo[o] = ok ? target[e] : 0.f;
    go[o] = ok && accumulate ? grad[e] : 0.f;
  }
  const float* src[3] = {abc, abc + n3, abc + 2 * n3};
  ssim_stage<3>(s, src, in);
  __syncthreads();
  ssim_hpass<3>(t.g, in, hs);
  __syncthreads();
  float m[kSsimBlk][3];
  ssim_vpass<3>(t.g, hs, r0, c, m);
  const float scale = -weight / (3.f * (float)s.W * (float)s.H);
#pragma unroll
  for (int o = 0; o < kSsimBlk; ++o) {
    const int gy = s.y0 + r0 + o;
    if (gx >= s.W || gy >= s.H) continue;
    const int64_t e = s.plane + (int64_t)gy * s.W + gx;
    const float g = scale * (m[o][0] + 2.f * xo[o] * m[o][1] + yo[o] * m[o][2]);
    grad[e] = accumulate ? go[o] + g : g;
  }
}

// Photometric seeds of the full training loss (eqs. 8 and 10), the D-SSIM gradient of
// k_ssim_grad plus the L1 terms: dL/dC = w_ssim dL_D-SSIM/dC + w_color sgn(C - Cbar) / (3 W H),
// dL/dD = w_depth [Dbar > 0] sgn(D - Dbar) / (W H) (channel-0 workgroups), and each workgroup's
// share of the weighted L1 loss in l1_partial.
__global__ __launch_bounds__(256) void k_photo_seeds(const float* __restrict__ color, const float* __restrict__ target,
                                                     const float* __restrict__ depth, const float* __restrict__ tdepth,
                                                     SsimTable t, const float* __restrict__ abc, int64_t n3,
                                                     float w_ssim, float w_color, float w_depth,
                                                     float* __restrict__ gcolor, float* __restrict__ gdepth,
                                                     double* __restrict__ l1_partial) {
  __shared__ __align__(16) float in[3][kSsimIH][kSsimLW];
  __shared__ float hs[3][kSsimIH][kSsimTW];
  __shared__ double red[4];
  const int b = ssim_block(t);
  if (b < 0) return;                       // whole workgroup
  const SsimTile s = ssim_tile(t, b);
  // this thread's outputs: rows r0 .. r0 + 3 of column c; their colour and depth values are
  // loaded first, so that their latency overlaps the staging
  const int c = threadIdx.x & (kSsimTW - 1), r0 = (threadIdx.x / kSsimTW) * kSsimBlk;
  const int gx = s.x0 + c;
  float xo[kSsimBlk], yo[kSsimBlk], dz[kSsimBlk], dt[kSsimBlk];
#pragma unroll
  for (int o = 0; o < kSsimBlk; ++o) {
    const int gy = s.y0 + r0 + o;
    const bool ok = gx < s.W && gy < s.H;
    const int64_t e = s.plane + (int64_t)gy * s.W + gx;
    const int64_t d = t.pix_off[s.v] + (int64_t)gy * s.W + gx;
    xo[o] = ok ? color[e] : 0.f;
    yo[o] = ok ? target[e] : 0.f;
    dz[o] = ok && s.ch == 0 ? depth[d] : 0.f;
    dt[o] = ok && s.ch == 0 ? tdepth[d] : 0.f;
  }
  const float* src[3] = {abc, abc + n3, abc + 2 * n3};
  ssim_stage<3>(s, src, in);
  __syncthreads();
  ssim_hpass<3>(t.g, in, hs);
  __syncthreads();
  float m[kSsimBlk][3];
  ssim_vpass<3>(t.g, hs, r0, c, m);
  const float npix = (float)s.W * (float)s.H;
  const float k_ssim = -w_ssim / (3.f * npix), k_col = w_color / (3.f * npix), k_dep = w_depth / npix;
  float l1 = 0.f;
#pragma unroll
  for (int o = 0; o < kSsimBlk; ++o) {
    const int gy = s.y0 + r0 + o;
    if (gx >= s.W || gy >= s.H) continue;
    const int64_t e = s.plane + (int64_t)gy * s.W + gx;
    const float x = xo[o], dc = x - yo[o];
    const float sg = (float)((dc > 0.f) - (dc < 0.f));
    gcolor[e] = k_ssim * (m[o][0] + 2.f * x * m[o][1] + yo[o] * m[o][2]) + k_col * sg;
    l1 += k_col * fabsf(dc);
    if (s.ch == 0) {
      const int64_t d = t.pix_off[s.v] + (int64_t)gy * s.W + gx;
      const float db = dt[o], dd = dz[o] - db;
      const bool valid = db > 0.f;
      gdepth[d] = valid ? k_dep * (float)((dd > 0.f) - (dd < 0.f)) : 0.f;
      if (valid) l1 += k_dep * fabsf(dd);
    }
  }
  double sum = (double)l1;
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) l1_partial[b] = (red[0] + red[1]) + (red[2] + red[3]);
}

// loss[v] = w_ssim (1 - sum of SSIM / (3 W H)) + the view's L1 partials (when given).
__global__ __launch_bounds__(1024) void k_ssim_loss(SsimTable t, const double* __restrict__ partial,
                                                    const double* __restrict__ l1_partial, float w_ssim,
                                                    float* __restrict__ loss) {
  __shared__ double red[2][16];
  const int v = blockIdx.x;
  double s4[4] = {0.0, 0.0, 0.0, 0.0}, l4[4] = {0.0, 0.0, 0.0, 0.0};
  const int b0 = t.blk_off[v], b1 = t.blk_off[v + 1];
  for (int b = b0 + threadIdx.x; b < b1; b += 4 * blockDim.x) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int bb = b + u * blockDim.x;
      if (bb < b1) {
        s4[u] += partial[bb];
        if (l1_partial) l4[u] += l1_partial[bb];
      }
    }
  }
  double sum = (s4[0] + s4[1]) + (s4[2] + s4[3]), l1 = (l4[0] + l4[1]) + (l4[2] + l4[3]);
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o, 64);
    l1 += __shfl_xor(l1, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sum;
    red[1][threadIdx.x >> 6] = l1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ss = 0.0, ll = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      ss += red[0][w];
      ll += red[1][w];
    }
    const double n = 3.0 * (double)t.width[v] * (double)t.height[v];
    loss[v] = (float)((double)w_ssim * (1.0 - ss / n) + ll);
  }
}

int build_ssim_table(const tsr_intrinsics* intr, int n_views, SsimTable* t) {
  if (!intr || n_views < 1 || n_views > TSR_MAX_VIEWS) return -1;
  memset(t, 0, sizeof *t);
  int64_t blocks = 0, pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = intr[v].width, H = intr[v].height;
    if (W <= 0 || H <= 0 || W > 16384 || H > 16384) return -1;
    t->width[v] = W;
    t->height[v] = H;
    t->tiles_x[v] = (W + kSsimTW - 1) / kSsimTW;
    t->tiles_y[v] = (H + kSsimTH - 1) / kSsimTH;
    t->pix_off[v] = pix;
    t->blk_off[v] = (int32_t)blocks;
    blocks += 3ll * t->tiles_x[v] * t->tiles_y[v];
    pix += (int64_t)W * H;
  }
  t->blk_off[n_views] = (int32_t)blocks;
  t->n_views = n_views;
  t->n_pixels = pix;
  // the 1-D factor of the Gaussian window, normalised in FP64
  double g[2 * kSsimR + 1], sum = 0.0;
  for (int k = 0; k < 2 * kSsimR + 1; ++k) {
    const double d = k - kSsimR;
    g[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[k];
  }
  for (int k = 0; k < 2 * kSsimR + 1; ++k) t->g[k] = (float)(g[k] / sum);
  return 0;
}

// Scratch layout: A, B, C maps [3][3P] | colour seeds [3P] | depth seeds [P] | SSIM partials
// [blocks] | L1 partials [blocks] (P = pixels of all views, each part 256-byte aligned).
struct SsimScratch {
  size_t abc, gcolor, gdepth, partial, l1_partial, total;
};

static SsimScratch ssim_scratch(const SsimTable& t) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t P = (size_t)t.n_pixels, nb = (size_t)t.blk_off[t.n_views];
  SsimScratch z;
  z.abc = 0;
  z.gcolor = up(z.abc + sizeof(float) * 9 * P);
  z.gdepth = up(z.gcolor + sizeof(float) * 3 * P);
  z.partial = up(z.gdepth + sizeof(float) * P);
  z.l1_partial = up(z.partial + sizeof(double) * nb);
  z.total = up(z.l1_partial + sizeof(double) * nb);
  return z;
}

size_t ssim_scratch_bytes(const SsimTable& t) { return ssim_scratch(t).total; }

hipError_t launch_dssim(const SsimTable& t, const float* color, const float* target, float weight,
                        bool accumulate, float* loss, float* grad, char* scratch, hipStream_t st) {
  const SsimScratch z = ssim_scratch(t);
  const int64_t n3 = 3 * t.n_pixels;
  float* abc = reinterpret_cast<float*>(scratch + z.abc);
  double* partial = reinterpret_cast<double*>(scratch + z.partial);
  TSR_LAUNCH("ssim_stats", k_ssim_stats, dim3(ssim_grid(t)), dim3(256), 0, st, color, target, t, abc, n3, partial);
  if (grad)
    TSR_LAUNCH("ssim_grad", k_ssim_grad, dim3(ssim_grid(t)), dim3(256), 0, st, color, target, t, abc, n3, weight,
               accumulate ? 1 : 0, grad);
  if (loss)
    TSR_LAUNCH("ssim_loss", k_ssim_loss, dim3(t.n_views), dim3(1024), 0, st, t, partial, (const double*)nullptr, 1.f,
               loss);
  return hipGetLastError();
}

hipError_t launch_photo_seeds(const SsimTable& t, const float* color, const float* target, const float* depth,
                              const float* tdepth, float w_ssim, float w_color, float w_depth, float* loss,
                              char* scratch, float** gcolor, float** gdepth, hipStream_t st) {
  const SsimScratch z = ssim_scratch(t);
  const int64_t n3 = 3 * t.n_pixels;
  float* abc = reinterpret_cast<float*>(scratch + z.abc);
  double* partial = reinterpret_cast<double*>(scratch + z.partial);
  double* l1_partial = reinterpret_cast<double*>(scratch + z.l1_partial);
  *gcolor = reinterpret_cast<float*>(scratch + z.gcolor);
  *gdepth = reinterpret_cast<float*>(scratch + z.gdepth);
  TSR_LAUNCH("ssim_stats", k_ssim_stats, dim3(ssim_grid(t)), dim3(256), 0, st, color, target, t, abc, n3, partial);
  TSR_LAUNCH("photo_seeds", k_photo_seeds, dim3(ssim_grid(t)), dim3(256), 0, st, color, target, depth, tdepth, t, abc, n3,
             w_ssim, w_color, w_depth, *gcolor, *gdepth, l1_partial);
  if (loss)
    TSR_LAUNCH("ssim_loss", k_ssim_loss, dim3(t.n_views), dim3(1024), 0, st, t, partial, (const double*)l1_partial,
               w_ssim, loss);
  return hipGetLastError();
}

}  // namespace tsr
