// Blend half of the hot path (gfx950): per-tile front-to-back compositing (eq. 4) of the
// window-weighted (eq. 3) barycentric colours and depths, its back-to-front backward pass,
// and the fused forward + L1 seeds + backward training kernel.
//
// Work mapping: one 256-lane workgroup per 16x16 tile, one pixel per lane; wave w owns the
// 8x8 quadrant (w & 1, w >> 1), so a face whose pixel rectangle misses a quadrant is skipped
// by that wave with one scalar test.  Face records are staged in LDS in batches of kBatch,
// loaded once per workgroup with coalesced 16-byte loads and read by all lanes as broadcasts.
#include "tsr_internal.h"

namespace tsr {

constexpr int kBatch = 64;                 // faces per hit mask (one lane each)
constexpr int kSpan = 256;                 // faces staged at once by a cooperative workgroup
constexpr int kSepSpan = 128;              // ... in the separate forward and backward kernels
constexpr int kWaves = kBlock / kWave;     // waves per workgroup: one per 8x8 quadrant

// Tiles whose list is longer than this many faces raise their wave priority (0 = off).  The
// longest tiles finish last; letting their waves win issue arbitration shortens the tail.
#ifndef TSR_PRIO_LONG
#define TSR_PRIO_LONG 240
#endif

// XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so give each XCD a
// contiguous range of tiles (neighbouring tiles share faces, which then hit the same L2).
__device__ __forceinline__ int tile_of_block(int n_tiles) {
  const int per = (n_tiles + 7) >> 3;
  const int idx = blockIdx.x >> 3;
  const int t = (int)(blockIdx.x & 7) * per + idx;
  return (idx < per && t < n_tiles) ? t : -1;
}

// Tile of a one-workgroup-per-tile launch: the longest-first order when one is given (the
// permutation of the tile ids built with the binning; an entry outside [0, n_tiles) gives no
// tile), else the XCD-interleaved id order.
__device__ __forceinline__ int tile_of_block_ordered(int n_tiles, const int* __restrict__ order) {
  if (!order) return tile_of_block(n_tiles);
  if ((int)blockIdx.x >= n_tiles) return -1;
  const int t = order[blockIdx.x];
  return (t >= 0 && t < n_tiles) ? t : -1;
}

// Kernel modes: the low three bits select the window exponent -- 1: sigma = 1, 2: sigma = 0.5,
// 3: sigma = 2, 0: any sigma, 4: each face's own sigma (from its record) -- and bit 3 the
// perspective-correct interpolation (numerator and denominator planes in the record).
template <int SM> constexpr int exp_mode() { return SM & 7; }
template <int SM> constexpr bool persp_mode() { return (SM & 8) != 0; }
// Bit 4: the separate forward and backward walks also composite each face's world normal (a
// colour constant over the face) into a normal map and back-propagate its seeds (mapping step).
template <int SM> constexpr bool normal_mode() { return (SM & 16) != 0; }

// Normal channels: per face, not per view, indexed by m = g - v M for the record slot
// g = v M + m.  The normal is a world quantity and its seeds are rotated into the world frame,
// so the gradients of all views add into one entry per face.
// The normal loss is evaluated where its inputs are: the forward rotates each pixel's
// composited normal into the camera frame (N = R_CW N_w), compares it with the target and
// leaves per-wave sums; the backward forms the seed dE/dN_w = R_CW^T dE/dN from the target and
// the view's valid-pixel count.
struct NormalIn {
  const float4* nrm;       // [M] unit world normal (x, y, z, 0)
  float4* gacc;            // backward: [M] dE/dn_F summed over the views (x, y, z, 0)
  float* map;              // forward, may be null: [sum 3 P] N in the camera frame, packed like colour
  const float* poses;      // [V][12] world-to-camera poses (row-major R, then t)
  const float* target;     // [sum 3 P] target normals, packed like colour (zero vector: invalid)
  const uint32_t* count;   // backward: [V] valid target pixels per view
  float* part;             // forward: [n_tiles * 4][8] per-wave sums (valid pixels, sum of
                           // 1 - N.N_bar, sum of N x N_bar)
  float w_norm;
  int64_t M;
};

// Window value for rho in (0, 1): I = rho^sigma (eq. 3).
template <int SM>
__device__ __forceinline__ float window_pow(float rho, float sigma) {
  if constexpr (exp_mode<SM>() == 1) return rho;
  else if constexpr (exp_mode<SM>() == 2) return __builtin_sqrtf(rho);
  else if constexpr (exp_mode<SM>() == 3) return rho * rho;
  else return exp2f(sigma * log2f(rho));
}

// The exponent a face is evaluated with: its record's in mode 4, else the launch's.
template <int SM>
__device__ __forceinline__ float face_sigma(const float* r, float sigma) {
  if constexpr (exp_mode<SM>() == 4) return r[kRecSigma];
  else return sigma;
}

struct PixelEval {
  float rho, I, alpha, c0, c1, c2;
  float zp;        // depth blended into D: z_F, or 1 / W (perspective-correct; then also 1 / W
                   // of the colour's numerators), 0 where the face does not cover the pixel
  bool k0, k1;     // the edge attaining the minimum of E_k is edge 0 / edge 1 (lowest index on
                   // ties; edge 2 when neither)
};

// A face record held in registers (loaded from LDS with six 16-byte reads).
struct Rec {
  float f[kRecDwords];
};

__device__ __forceinline__ void load_rec(const float4* srec, int j, Rec& r) {
#pragma unroll
  for (int i = 0; i < kRecDwords / 4; ++i) {
    const float4 q = srec[j * 6 + i];
    r.f[4 * i] = q.x;
    r.f[4 * i + 1] = q.y;
    r.f[4 * i + 2] = q.z;
    r.f[4 * i + 3] = q.w;
  }
}

// Evaluates one face at face-local pixel offset (dx, dy), without branches; returns whether
// the pixel is covered (rho > 0 and alpha > 0).  alpha and I are zero when it is not.
// Identical instructions in the forward and backward walks, so the backward recomputes
// alpha bit for bit.
template <int SM>
__device__ __forceinline__ bool eval_face(const Rec& rc, float dx, float dy, float sigma, PixelEval& e) {
  const float* r = rc.f;
  const float E0 = fmaf(r[kRecEdge + 0], dx, fmaf(r[kRecEdge + 1], dy, r[kRecEdge + 2]));
  const float E1 = fmaf(r[kRecEdge + 3], dx, fmaf(r[kRecEdge + 4], dy, r[kRecEdge + 5]));
  const float E2 = fmaf(r[kRecEdge + 6], dx, fmaf(r[kRecEdge + 7], dy, r[kRecEdge + 8]));
  e.k0 = E0 <= E1 && E0 <= E2;
  e.k1 = !e.k0 && E1 <= E2;
  e.rho = fminf(E0, fminf(E1, E2));
  const float I = e.rho >= 1.f ? 1.f : window_pow<SM>(e.rho, face_sigma<SM>(r, sigma));   // meaningless when rho <= 0
  const float alpha = r[kRecOpa] * I;
  const bool cov = e.rho > 0.f && alpha > 0.f;
  e.I = cov ? I : 0.f;
  e.alpha = cov ? alpha : 0.f;
  e.c0 = fmaf(r[kRecCol + 0], dx, fmaf(r[kRecCol + 1], dy, r[kRecCol + 2]));
  e.c1 = fmaf(r[kRecCol + 3], dx, fmaf(r[kRecCol + 4], dy, r[kRecCol + 5]));
  e.c2 = fmaf(r[kRecCol + 6], dx, fmaf(r[kRecCol + 7], dy, r[kRecCol + 8]));
  if constexpr (persp_mode<SM>()) {
    // colour = numerator planes / W and depth = 1 / W (W > 0 where the face covers the pixel;
    // elsewhere the weight is 0 and so is 1 / W here)
    const float W = fmaf(r[kRecWa], dx, fmaf(r[kRecWb], dy, r[kRecWc]));
    const float iW = cov ? __builtin_amdgcn_rcpf(W) : 0.f;
    e.c0 *= iW;
    e.c1 *= iW;
    e.c2 *= iW;
    e.zp = iW;
  } else {
    e.zp = r[kRecZ];
  }
  return cov;
}

// Geometry of this lane's pixel inside the tile.
struct TileCtx {
  int tile, view;
  ViewDesc vd;
  int bx, by;            // top-left pixel of this wave's 8x8 quadrant
  int px, py;
  bool inside;
  int64_t pix;           // packed pixel index (valid when inside)
  uint32_t start, end;   // tile list range
};

__device__ __forceinline__ void tile_ctx(const ViewTable& vt, const uint32_t* __restrict__ ranges, int tile,
                                         int quad, TileCtx& c) {
  c.tile = tile;
  c.view = view_of_tile(vt, tile);
  c.vd = vt.v[c.view];
  const int lt = tile - c.vd.tile_off;
  const int tx = lt % c.vd.tiles_x, ty = lt / c.vd.tiles_x;
  const int lane = threadIdx.x & 63;
  c.bx = tx * kTile + (quad & 1) * 8;
  c.by = ty * kTile + (quad >> 1) * 8;
  c.px = c.bx + (lane & 7);
  c.py = c.by + (lane >> 3);
  c.inside = c.px < c.vd.width && c.py < c.vd.height;
  c.pix = c.vd.pix_off + (int64_t)c.py * c.vd.width + c.px;
  c.start = ranges[2 * tile];
  c.end = ranges[2 * tile + 1];
}

// Makes this wave's LDS stores visible to its own later loads from other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Two ways to stage the records of pair positions [b0, b0 + n), n <= kBatch, into LDS:
//  * cooperative (COOP): the four waves of the workgroup load one shared copy, with a barrier
//    before and after, so all waves walk the batches in step (one copy of the records per
//    tile is read from the caches);
//  * per wave: each wave loads its own copy into its own LDS area and walks the list at its
//    own pace (no barriers; four copies are read).
// Which one is faster depends on how often the caches already hold the records.
// Cooperative kernels always run kBlock threads; the staging loops below stride by kBlock, so
// a span of any length up to kSpan is staged completely (every entry's face id and record).
static_assert(kSpan % kBatch == 0 && kSpan >= kBatch, "a staged span is walked as whole 64-face batches");
static_assert(kSepSpan % kBatch == 0 && kSepSpan >= kBatch && kSepSpan <= kSpan, "as kSpan");
static_assert(kSpan * (6 * sizeof(float4) + sizeof(uint32_t)) <= 48 * 1024, "a staged span fits the LDS budget");
static_assert(kWaves * kWave == kBlock && kWaves == 4, "one wave per 8x8 quadrant of a 16x16 tile");
static_assert(kGradDwords == 20, "normal channels: record terms in slots 0-19 of the 24-value wave sum");
static_assert(kWaves == kTileQuads, "normal-loss sums: one slot per wave of a tile");
__device__ __forceinline__ void stage_batch_block(const float* __restrict__ records, const uint64_t* __restrict__ pairs,
                                                  uint32_t b0, int n, float4* srec, uint32_t* sface,
                                                  const float4* __restrict__ nrm = nullptr, int64_t moff = 0,
                                                  float4* snrm = nullptr) {
  for (int i = threadIdx.x; i < n * 6; i += kBlock) {
    const uint32_t face = (uint32_t)pairs[b0 + i / 6];
    srec[i] = reinterpret_cast<const float4*>(records)[(size_t)face * 6 + i % 6];
  }
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const uint32_t face = (uint32_t)pairs[b0 + i];
    sface[i] = face;
    if (nrm) snrm[i] = nrm[(int64_t)face - moff];
  }
}

// Per-wave staging: lane l reads the face id of entry l; the 6 n sixteen-byte pieces are then
// loaded by the lanes in turn (piece i by lane i % 64, face id taken from lane i / 6).  With
// the normal channels, lane l also stages the normal of face l into snrm.
__device__ __forceinline__ void stage_batch(const float* __restrict__ records, const uint64_t* __restrict__ pairs,
                                            uint32_t b0, int n, float4* srec, uint32_t* sface,
                                            const float4* __restrict__ nrm = nullptr, int64_t moff = 0,
                                            float4* snrm = nullptr) {
  const int lane = threadIdx.x & 63;
  const uint32_t f = lane < n ? (uint32_t)pairs[b0 + lane] : 0u;
  if (lane < n) sface[lane] = f;
  if (nrm && lane < n) snrm[lane] = nrm[(int64_t)f - moff];
  const float4* rec4 = reinterpret_cast<const float4*>(records);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int i = lane + 64 * k;
    const uint32_t fi = (uint32_t)__shfl((int)f, i / 6, 64);
    if (i < n * 6) srec[i] = rec4[(size_t)fi * 6 + i % 6];
  }
  wave_lds_sync();
}

// Faces of the staged batch that can cover a pixel of this wave's 8x8 quadrant: lane j tests
// face j, one ballot gives the wave-uniform 64-bit mask the walks iterate over.  A face is
// kept when its pixel rectangle meets the quadrant and no edge function is negative over the
// whole intersection box: the maximum of E_k = a dx + b dy + c over the box is at one of its
// corners, and a face with that maximum below -margin has rho <= 0 (no blend, zero gradient)
// at every pixel the walks would evaluate, so skipping it changes nothing.  The margin (1e-6 of
// the magnitude of the terms) exceeds the FP32 rounding of both evaluations.
// Perspective-correct records do not hold the rectangle's end: the edge test then runs over
// the whole quadrant (still conservative).
template <int SM>
__device__ __forceinline__ unsigned long long batch_hit_mask(const float4* srec, int n, int bx, int by) {
  const int j = threadIdx.x & 63;
  bool hit = false;
  if constexpr (persp_mode<SM>()) {
    if (j < n) {
      const float4 rc = srec[j * 6 + kRecU0 / 4];
      const float* r = reinterpret_cast<const float*>(&srec[j * 6]);
      const float dxl = (float)bx - rc.x, dxh = (float)(bx + 7) - rc.x;
      const float dyl = (float)by - rc.y, dyh = (float)(by + 7) - rc.y;
      const float mx = fmaxf(fabsf(dxl), fabsf(dxh)), my = fmaxf(fabsf(dyl), fabsf(dyh));
      hit = true;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float a = r[kRecEdge + 3 * k], b = r[kRecEdge + 3 * k + 1], c = r[kRecEdge + 3 * k + 2];
        const float dx = a > 0.f ? dxh : dxl, dy = b > 0.f ? dyh : dyl;
        const float emax = fmaf(a, dx, fmaf(b, dy, c));
        const float margin = 1e-6f * (fabsf(a) * mx + fabsf(b) * my + fabsf(c)) + 1e-30f;
        hit = hit && !(emax < -margin);
      }
    }
    return ballot(hit);
  }
  if (j < n) {
    const float4 rc = srec[j * 6 + kRecU0 / 4];
    const int u1v1 = __float_as_int(rc.z);
    const int u0 = (int)rc.x, v0 = (int)rc.y, u1 = u1v1 & 0xffff, v1 = u1v1 >> 16;
    const int xl = max(bx, u0), xh = min(bx + 7, u1), yl = max(by, v0), yh = min(by + 7, v1);
    hit = xl <= xh && yl <= yh;
    if (hit) {
      const float* r = reinterpret_cast<const float*>(&srec[j * 6]);
      const float dxl = (float)(xl - u0), dxh = (float)(xh - u0), dyl = (float)(yl - v0), dyh = (float)(yh - v0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float a = r[kRecEdge + 3 * k], b = r[kRecEdge + 3 * k + 1], c = r[kRecEdge + 3 * k + 2];
        const float dx = a > 0.f ? dxh : dxl, dy = b > 0.f ? dyh : dyl;
        const float emax = fmaf(a, dx, fmaf(b, dy, c));
        const float margin = 1e-6f * (fabsf(a) * dxh + fabsf(b) * dyh + fabsf(c)) + 1e-30f;
        hit = hit && !(emax < -margin);
      }
    }
  }
  return ballot(hit);
}

struct FwdState {
  float T, C0, C1, C2, D, Tb;
  float N0, N1, N2;        // composited world normal (normal channels)
  int last;
};

// A pixel blends faces while its transmittance is at least t_min and positive.  T never
// increases, so this is the rule "stop after the face that takes T below t_min, or to 0"
// (t_min < 1) without a separate state; pixels outside the image start at T = 0.  One
// comparison against max(t_min, FLT_MIN) (hoisted by the compiler) tests both: the two differ
// only for t_min = 0 at a subnormal T, where nothing visible is left to blend.
__device__ __forceinline__ bool live(float T, float t_min) { return T >= fmaxf(t_min, 1.17549435e-38f); }

// Front-to-back walk over the tile list (eq. 4).  A pixel stops after the face that takes
// its transmittance below t_min.  Records each pixel's last blended face and the
// transmittance just before it.
template <int SM, bool COOP, int SPAN = kSpan>
__device__ __forceinline__ void forward_walk(const TileCtx& c, const float* __restrict__ records,
                                             const uint64_t* __restrict__ pairs, float sigma, float t_min,
                                             float4* srec, uint32_t* sface, FwdState& s,
                                             const NormalIn* nin = nullptr, float4* snrm = nullptr) {
  s.T = c.inside ? 1.f : 0.f;
  s.C0 = s.C1 = s.C2 = s.D = 0.f; s.Tb = 1.f; s.last = -1;
  s.N0 = s.N1 = s.N2 = 0.f;
  const float dxb = (float)c.px, dyb = (float)c.py;
  constexpr int kStage = COOP ? SPAN : kBatch;      // faces staged at once
  for (uint32_t s0 = c.start; s0 < c.end; s0 += kStage) {
    const int ns = (int)min((uint32_t)kStage, c.end - s0);
    if constexpr (COOP) {
      if (__syncthreads_count(live(s.T, t_min)) == 0) break;
      if constexpr (normal_mode<SM>())
        stage_batch_block(records, pairs, s0, ns, srec, sface, nin->nrm, (int64_t)c.view * nin->M, snrm);
      else
        stage_batch_block(records, pairs, s0, ns, srec, sface);
      __syncthreads();
    } else {
      if (ballot(live(s.T, t_min)) == 0) break;
      if constexpr (normal_mode<SM>())
        stage_batch(records, pairs, s0, ns, srec, sface, nin->nrm, (int64_t)c.view * nin->M, snrm);
      else
        stage_batch(records, pairs, s0, ns, srec, sface);
    }
    for (int h = 0; h < ns; h += kBatch) {
    bool lv = live(s.T, t_min);         // this lane still blends (carried across the visits)
    if (ballot(lv) == 0) break;
    const int n = min(kBatch, ns - h);
    const uint32_t b0 = s0 + (uint32_t)h;
    const float4* sr = srec + h * 6;
    unsigned long long mask = batch_hit_mask<SM>(sr, n, c.bx, c.by);
    while (mask) {
      const int j = __builtin_ctzll(mask);
      mask &= mask - 1;
      Rec rc;
      load_rec(sr, j, rc);
      PixelEval e;
      const float dx = dxb - rc.f[kRecU0];
      const float dy = dyb - rc.f[kRecV0];
      // stopping also at T == 0 means the backward never divides by 1 - alpha = 0
      const bool act = eval_face<SM>(rc, dx, dy, sigma, e) && lv;
      // lanes that do not blend this face keep their state: alpha 0 gives weight 0 and T * 1
      const float a = act ? e.alpha : 0.f;
      const float w = a * s.T;
      s.C0 = fmaf(e.c0, w, s.C0);
      s.C1 = fmaf(e.c1, w, s.C1);
      s.C2 = fmaf(e.c2, w, s.C2);
      s.D = fmaf(e.zp, w, s.D);
      if constexpr (normal_mode<SM>()) {
        const float4 nf = snrm[h + j];
        s.N0 = fmaf(nf.x, w, s.N0);
        s.N1 = fmaf(nf.y, w, s.N1);
        s.N2 = fmaf(nf.z, w, s.N2);
      }
      s.Tb = act ? s.T : s.Tb;
      s.last = act ? (int)(b0 + j) : s.last;
      s.T = s.T * (1.f - a);
      lv = live(s.T, t_min);
      if (ballot(lv) == 0) break;
    }
    }
  }
}

// Per-pixel upstream gradients (gn: of the world normal map, normal channels).
struct PixGrad {
  float g0, g1, g2, gd, gt;
  float gn0 = 0.f, gn1 = 0.f, gn2 = 0.f;
};

// Back-to-front walk (Sec. 3.3).  T before each face is recovered by division from the
// transmittance before the last blended face.  What lies behind the current face, composited
// from transmittance 1 (colour B, depth BD, opacity BA), enters dL/dalpha only through
// S = gC.B + gD BD - gT BA, so S is carried instead: with P = gC.c + gD z - gT for the face,
// dL/dalpha = T (P - S) and S <- alpha P + (1 - alpha) S.  Per-face sums of the 20
// record-parameter gradients are reduced over the wave and added to grad_acc.
template <int SM, bool COOP, int SPAN = kSpan>
__device__ __forceinline__ void backward_walk(const TileCtx& c, const float* __restrict__ records,
                                              const uint64_t* __restrict__ pairs, float sigma, int last, float Tb,
                                              const PixGrad& pg, float4* srec, uint32_t* sface, int* sint,
                                              acc_t* __restrict__ grad_acc, float* __restrict__ sig_acc,
                                              float* __restrict__ persp_acc, const NormalIn* nin = nullptr,
                                              float4* snrm = nullptr) {
  const int lane = threadIdx.x & 63;
  // highest list position any pixel of this wave (COOP: of the workgroup) blended
  const int wlast = uniform_int(wave_max_int(last));
  int top = wlast;
  if constexpr (COOP) {
    if (threadIdx.x == 0) sint[0] = -1;
    __syncthreads();
    if (lane == 0) atomicMax(&sint[0], wlast);
    __syncthreads();
    top = uniform_int(sint[0]);
  }
  // With terms beyond the record's 20 (normal channels: 3 in slots 20-22; perspective without
  // them: the W plane's 2 slopes in slots 20-21; per-face exponent: slot 23) all go through one
  // 24-value transposed sum.
  constexpr bool kWide = normal_mode<SM>() || persp_mode<SM>() || exp_mode<SM>() == 4;
  const int k_out = kWide ? wave_sum24_slot() : wave_sum20_slot();
  float Tcur = Tb;
  float S = 0.f;
  const float dxb = (float)c.px, dyb = (float)c.py;
  constexpr int kStage = COOP ? SPAN : kBatch;      // faces staged at once
  for (int s1 = top + 1; s1 > (int)c.start; s1 -= kStage) {
    const int s0 = max((int)c.start, s1 - kStage);
    const int ns = s1 - s0;
    if constexpr (COOP) {
      __syncthreads();
      if constexpr (normal_mode<SM>())
        stage_batch_block(records, pairs, (uint32_t)s0, ns, srec, sface, nin->nrm, (int64_t)c.view * nin->M, snrm);
      else
        stage_batch_block(records, pairs, (uint32_t)s0, ns, srec, sface);
      __syncthreads();
    } else {
      if constexpr (normal_mode<SM>())
        stage_batch(records, pairs, (uint32_t)s0, ns, srec, sface, nin->nrm, (int64_t)c.view * nin->M, snrm);
      else
        stage_batch(records, pairs, (uint32_t)s0, ns, srec, sface);
    }
    for (int h = ((ns - 1) / kBatch) * kBatch; h >= 0; h -= kBatch) {
    const int b0 = s0 + h;
    const int n = min(kBatch, ns - h);
    if (b0 > wlast) continue;
    const float4* sr = srec + h * 6;
    const uint32_t* sf = sface + h;
    unsigned long long mask = batch_hit_mask<SM>(sr, n, c.bx, c.by);
    if (wlast - b0 < 63) mask &= (2ull << (wlast - b0)) - 1ull;     // faces after the wave's last
    while (mask) {
      const int j = 63 - __builtin_clzll(mask);
      mask &= ~(1ull << j);
      const int idx = b0 + j;
      Rec rc;
      load_rec(sr, j, rc);
      const float* r = rc.f;
      // Every lane evaluates the face; lanes that do not blend it (not covered, or behind
      // their last face) get alpha = I = 0, hence zero weight and zero gradient scales, so
      // all 20 sums need no branches.
      const float dx = dxb - r[kRecU0];
      const float dy = dyb - r[kRecV0];
      PixelEval e;
      const bool act = eval_face<SM>(rc, dx, dy, sigma, e) && (idx <= last);
      const float alpha = act ? e.alpha : 0.f;
      const float I = act ? e.I : 0.f;
      const float om = 1.f - alpha;
      // T before this face: the stored value at the last face, else T_after / (1 - alpha)
      const float Tj = (idx == last) ? Tb : Tcur * __builtin_amdgcn_rcpf(om);
      Tcur = act ? Tj : Tcur;
      const float zf = e.zp;
      const float c0 = e.c0, c1 = e.c1, c2 = e.c2;
      const float w = alpha * Tj;
      float acc[kWide ? 24 : kGradDwords];
      // colour plane gradients: dL/dc_ch(p) = gC_ch alpha T, and c_ch = P dx + Q dy + R
      float gc0 = pg.g0 * w, gc1 = pg.g1 * w, gc2 = pg.g2 * w;
      float gwa = 0.f, gwb = 0.f;          // perspective-correct: the W plane's slopes
      if constexpr (persp_mode<SM>()) {
        // c_ch = N_ch / W, depth = 1 / W: dL/dN_ch = gC_ch w / W, dL/dW = -(gC.c + gD depth) w / W
        const float gW = -(fmaf(pg.g0, c0, fmaf(pg.g1, c1, fmaf(pg.g2, c2, pg.gd * zf)))) * w * zf;
        gc0 *= zf;
        gc1 *= zf;
        gc2 *= zf;
        acc[kGWc] = gW;
        gwa = gW * dx;
        gwb = gW * dy;
      } else {
        acc[kGZ] = pg.gd * w;
      }
      acc[kGCol + 0] = gc0 * dx; acc[kGCol + 1] = gc0 * dy; acc[kGCol + 2] = gc0;
      acc[kGCol + 3] = gc1 * dx; acc[kGCol + 4] = gc1 * dy; acc[kGCol + 5] = gc1;
      acc[kGCol + 6] = gc2 * dx; acc[kGCol + 7] = gc2 * dy; acc[kGCol + 8] = gc2;
      // dL/dalpha = T (gC.(c - B) + gD (z - BD) - gT (1 - BA)) = T (P - S); finite on every
      // lane, and only used scaled by I or masked by act
      float P = fmaf(pg.g0, c0, fmaf(pg.g1, c1, fmaf(pg.g2, c2, fmaf(pg.gd, zf, -pg.gt))));
      float4 nf = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (normal_mode<SM>()) {
        // the face's normal is a colour constant over the face: it enters dL/dalpha like one
        nf = snrm[h + j];
        P = fmaf(pg.gn0, nf.x, fmaf(pg.gn1, nf.y, fmaf(pg.gn2, nf.z, P)));
      }
      const float galpha = Tj * (P - S);
      acc[kGOpa] = galpha * I;
      const float gI = galpha * r[kRecOpa];
      float grho = 0.f;
      if constexpr (exp_mode<SM>() == 1) grho = (act && e.rho < 1.f) ? gI : 0.f;
      else grho = (act && e.rho < 1.f) ? gI * face_sigma<SM>(r, sigma) * I * __builtin_amdgcn_rcpf(e.rho) : 0.f;   // sigma I / rho
      // only the edge attaining the minimum receives the window gradient
      const float gk[3] = {e.k0 ? grho : 0.f, e.k1 ? grho : 0.f, (e.k0 || e.k1) ? 0.f : grho};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        acc[kGEdge + 3 * k + 0] = gk[k] * dx;
        acc[kGEdge + 3 * k + 1] = gk[k] * dy;
        acc[kGEdge + 3 * k + 2] = gk[k];
      }
      S = fmaf(alpha, P, om * S);
      if (ballot(act) == 0) continue;
      // the face's own exponent: dI/dsigma = I ln(rho) for 0 < rho < 1 (act implies rho > 0)
      float gsig = 0.f;
      if constexpr (exp_mode<SM>() == 4)
        gsig = (act && e.rho < 1.f) ? gI * I * (0.69314718055994531f * log2f(e.rho)) : 0.f;
      if constexpr (kWide) {
        if constexpr (normal_mode<SM>()) {
          // dE/dn_F = sum over the face's pixels of gN alpha T
          acc[20] = pg.gn0 * w;
          acc[21] = pg.gn1 * w;
          acc[22] = pg.gn2 * w;
        } else {
          acc[20] = gwa;
          acc[21] = gwb;
          acc[22] = 0.f;
        }
        acc[23] = gsig;
        const float tot = wave_sum24(acc);
        if (k_out >= 0 && k_out < kGradDwords) {
          unsafeAtomicAdd(&grad_acc[(size_t)sf[j] * kGradDwords + k_out], (acc_t)tot);
        } else if (normal_mode<SM>() && k_out >= kGradDwords && k_out < 23) {
          float* ga = reinterpret_cast<float*>(nin->gacc + ((int64_t)sf[j] - (int64_t)c.view * nin->M));
          unsafeAtomicAdd(&ga[k_out - kGradDwords], tot);
        } else if (!normal_mode<SM>() && persp_mode<SM>() && (k_out == 20 || k_out == 21)) {
          unsafeAtomicAdd(&persp_acc[2 * (size_t)sf[j] + (k_out - 20)], tot);
        } else if (exp_mode<SM>() == 4 && k_out == 23) {
          unsafeAtomicAdd(&sig_acc[sf[j]], tot);
        }
        if constexpr (normal_mode<SM>() && persp_mode<SM>()) {
          const float ta = wave_sum(gwa), tb = wave_sum(gwb);
          if (lane == 0) {
            unsafeAtomicAdd(&persp_acc[2 * (size_t)sf[j]], ta);
            unsafeAtomicAdd(&persp_acc[2 * (size_t)sf[j] + 1], tb);
          }
        }
      } else {
        const float tot = wave_sum20(acc);
        if (k_out >= 0) unsafeAtomicAdd(&grad_acc[(size_t)sf[j] * kGradDwords + k_out], (acc_t)tot);
      }
    }
    }
  }
}

// ---------------------------------------------------------------------------- kernels

// COOP: the tile's list is staged cooperatively (one shared copy per workgroup, the four
// quadrant waves in step), else per wave (four copies, each wave at its own pace).
template <int SM, bool COOP>
__global__ __launch_bounds__(kBlock) void k_blend_fwd(ViewTable vt, const float* __restrict__ records,
                                                      const uint64_t* __restrict__ pairs,
                                                      const uint32_t* __restrict__ ranges, float sigma, float t_min,
                                                      float* __restrict__ color, float* __restrict__ depth,
                                                      float* __restrict__ trans, int* __restrict__ n_last,
                                                      float* __restrict__ t_last, const int* __restrict__ order,
                                                      NormalIn nin) {
  const int wv = threadIdx.x >> 6;
  const int tile = tile_of_block_ordered(vt.n_tiles, order);
  if (tile < 0) return;
  TileCtx c;
  tile_ctx(vt, ranges, tile, wv, c);
  FwdState s;
  if constexpr (COOP) {
    __shared__ float4 srec[kSepSpan * 6];
    __shared__ uint32_t sface[kSepSpan];
    __shared__ float4 snrm[normal_mode<SM>() ? kSepSpan : 1];
    forward_walk<SM, true, kSepSpan>(c, records, pairs, sigma, t_min, srec, sface, s, &nin, snrm);
  } else {
    __shared__ float4 srec[kWaves][kBatch * 6];
    __shared__ uint32_t sface[kWaves][kBatch];
    __shared__ float4 snrm[kWaves][normal_mode<SM>() ? kBatch : 1];
    forward_walk<SM, false>(c, records, pairs, sigma, t_min, srec[wv], sface[wv], s, &nin, snrm[wv]);
  }
  const int64_t hw = (int64_t)c.vd.width * c.vd.height;
  const int64_t off = (int64_t)c.py * c.vd.width + c.px;
  if constexpr (normal_mode<SM>()) {
    // N = R_CW N_w against the target (Sec. 3.4); the wave's sums go to part (all lanes active)
    const float* R = nin.poses + 12 * c.view;
    const float n0 = R[0] * s.N0 + R[1] * s.N1 + R[2] * s.N2;
    const float n1 = R[3] * s.N0 + R[4] * s.N1 + R[5] * s.N2;
    const float n2 = R[6] * s.N0 + R[7] * s.N1 + R[8] * s.N2;
    float cnt = 0.f, l = 0.f, r0 = 0.f, r1 = 0.f, r2 = 0.f;
    if (c.inside) {
      const float* tb = nin.target + 3 * c.vd.pix_off + off;
      const float b0 = tb[0], b1 = tb[hw], b2 = tb[2 * hw];
      if (b0 != 0.f || b1 != 0.f || b2 != 0.f) {
        cnt = 1.f;
        l = 1.f - (n0 * b0 + n1 * b1 + n2 * b2);
        r0 = n1 * b2 - n2 * b1;
        r1 = n2 * b0 - n0 * b2;
        r2 = n0 * b1 - n1 * b0;
      }
      if (nin.map) {
        float* nb = nin.map + 3 * c.vd.pix_off + off;
        nb[0] = n0;
        nb[hw] = n1;
        nb[2 * hw] = n2;
      }
    }
    const float tc = wave_sum(cnt), tl = wave_sum(l), t0 = wave_sum(r0), t1 = wave_sum(r1), t2 = wave_sum(r2);
    if ((threadIdx.x & 63) == 0) {
      float4* pw = reinterpret_cast<float4*>(nin.part + kNormalPart * ((int64_t)tile * kWaves + wv));
      pw[0] = make_float4(tc, tl, t0, t1);
      pw[1] = make_float4(t2, 0.f, 0.f, 0.f);
    }
  }
  if (!c.inside) return;
  float* cb = color + 3 * c.vd.pix_off + off;
  cb[0] = s.C0;
  cb[hw] = s.C1;
  cb[2 * hw] = s.C2;
  depth[c.pix] = s.D;
  if (trans) trans[c.pix] = s.T;
  n_last[c.pix] = s.last;
  t_last[c.pix] = s.Tb;
}

template <int SM, bool COOP>
__global__ __launch_bounds__(kBlock) void k_blend_bwd(ViewTable vt, const float* __restrict__ records,
                                                      const uint64_t* __restrict__ pairs,
                                                      const uint32_t* __restrict__ ranges, float sigma,
                                                      const int* __restrict__ n_last, const float* __restrict__ t_last,
                                                      const float* __restrict__ gcolor, const float* __restrict__ gdepth,
                                                      const float* __restrict__ gtrans, acc_t* __restrict__ grad_acc,
                                                      float* __restrict__ sig_acc, float* __restrict__ persp_acc,
                                                      const int* __restrict__ order, NormalIn nin) {
  const int wv = threadIdx.x >> 6;
  const int tile = tile_of_block_ordered(vt.n_tiles, order);
  if (tile < 0) return;
  TileCtx c;
  tile_ctx(vt, ranges, tile, wv, c);
  int last = -1;
  float Tb = 0.f;
  PixGrad pg{0.f, 0.f, 0.f, 0.f, 0.f};
  if (c.inside) {
    last = n_last[c.pix];
    Tb = t_last[c.pix];
    // state from a forward over another binning must not index outside this tile's list
    if (last < (int)c.start || last >= (int)c.end) last = -1;
    const int64_t hw = (int64_t)c.vd.width * c.vd.height;
    const float* gb = gcolor + 3 * c.vd.pix_off + (int64_t)c.py * c.vd.width + c.px;
    pg.g0 = gb[0];
    pg.g1 = gb[hw];
    pg.g2 = gb[2 * hw];
    pg.gd = gdepth[c.pix];
    pg.gt = gtrans ? gtrans[c.pix] : 0.f;
    if constexpr (normal_mode<SM>()) {
      // dE/dN = -(w_norm / valid count) N_bar at a valid pixel, then dE/dN_w = R_CW^T dE/dN
      const float* tb = nin.target + 3 * c.vd.pix_off + (int64_t)c.py * c.vd.width + c.px;
      const float b0 = tb[0], b1 = tb[hw], b2 = tb[2 * hw];
      const uint32_t cn = nin.count[c.view];
      const float inv = cn ? nin.w_norm / (float)cn : 0.f;
      float g0 = 0.f, g1 = 0.f, g2 = 0.f;
      if (b0 != 0.f || b1 != 0.f || b2 != 0.f) {
        g0 = -inv * b0;
        g1 = -inv * b1;
        g2 = -inv * b2;
      }
      const float* R = nin.poses + 12 * c.view;
      pg.gn0 = R[0] * g0 + R[3] * g1 + R[6] * g2;
      pg.gn1 = R[1] * g0 + R[4] * g1 + R[7] * g2;
      pg.gn2 = R[2] * g0 + R[5] * g1 + R[8] * g2;
    }
  }
  if constexpr (COOP) {
    __shared__ float4 srec[kSepSpan * 6];
    __shared__ uint32_t sface[kSepSpan];
    __shared__ float4 snrm[normal_mode<SM>() ? kSepSpan : 1];
    __shared__ int sint[4];
    backward_walk<SM, true, kSepSpan>(c, records, pairs, sigma, last, Tb, pg, srec, sface, sint, grad_acc, sig_acc,
                                      persp_acc, &nin, snrm);
  } else {
    __shared__ float4 srec[kWaves][kBatch * 6];
    __shared__ uint32_t sface[kWaves][kBatch];
    __shared__ float4 snrm[kWaves][normal_mode<SM>() ? kBatch : 1];
    backward_walk<SM, false>(c, records, pairs, sigma, last, Tb, pg, srec[wv], sface[wv], nullptr, grad_acc, sig_acc,
                             persp_acc, &nin, snrm[wv]);
  }
}

// Fused training kernel: forward walk, L1 seeds of eqs. 8-10 (the D-SSIM term needs whole
// images and runs in tsr_ssim.hip between a separate forward and backward), backward
// walk, without leaving the workgroup.  Also writes the loss of each (tile, quadrant).
template <int SM>
__global__ __launch_bounds__(kBlock) void k_train_fused(ViewTable vt, const float* __restrict__ records,
                                                        const uint64_t* __restrict__ pairs,
                                                        const uint32_t* __restrict__ ranges, float sigma, float t_min,
                                                        float w_color, float w_depth,
                                                        const float* __restrict__ tcolor, const float* __restrict__ tdepth,
                                                        float* __restrict__ color, float* __restrict__ depth,
                                                        float* __restrict__ trans, float* __restrict__ loss_part,
                                                        acc_t* __restrict__ grad_acc, float* __restrict__ sig_acc,
                                                        float* __restrict__ persp_acc,
                                                        const int* __restrict__ order, int* __restrict__ queue,
                                                        int persistent) {
  // the four waves stage each span together (one copy of the records per tile)
  __shared__ float4 srec[kSpan * 6];
  __shared__ uint32_t sface[kSpan];
  __shared__ int s_item;
  __shared__ int sint[4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int round = 0;
  for (;;) {
    int tile;
    const int quad = wv;
    if (persistent) {
      // the workgroup's first tile is its own id; later ones come from the queue (items
      // gridDim.x onward), so the launch does not start with gridDim.x atomics on one address
      int item = (int)blockIdx.x;
      if (round > 0) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)gridDim.x + atomicAdd(queue, 1);
        __syncthreads();
        item = s_item;
      }
      ++round;
      if (item >= vt.n_tiles) break;
      tile = order ? order[item] : item;
    } else {
      tile = order ? ((int)blockIdx.x < vt.n_tiles ? order[blockIdx.x] : -1) : tile_of_block(vt.n_tiles);
      if (tile < 0) break;
    }
    TileCtx c;
    tile_ctx(vt, ranges, tile, quad, c);
#if TSR_PRIO_LONG
    // long tile lists bound the kernel's tail: let their waves win issue arbitration
    if (c.end - c.start > TSR_PRIO_LONG) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(0);
#endif
    FwdState s;
    forward_walk<SM, true>(c, records, pairs, sigma, t_min, srec, sface, s);
    PixGrad pg{0.f, 0.f, 0.f, 0.f, 0.f};
    float lpix = 0.f;
    if (c.inside) {
      const int64_t hw = (int64_t)c.vd.width * c.vd.height;
      const int64_t off = (int64_t)c.py * c.vd.width + c.px;
      const float inv_c = w_color / (3.f * (float)hw), inv_d = w_depth / (float)hw;
      const float* tc = tcolor + 3 * c.vd.pix_off + off;
      const float r0 = s.C0 - tc[0], r1 = s.C1 - tc[hw], r2 = s.C2 - tc[2 * hw];
      const float td = tdepth[c.pix];
      const float rd = s.D - td;
      const float md = td > 0.f ? 1.f : 0.f;
      pg.g0 = inv_c * (float)((r0 > 0.f) - (r0 < 0.f));
      pg.g1 = inv_c * (float)((r1 > 0.f) - (r1 < 0.f));
      pg.g2 = inv_c * (float)((r2 > 0.f) - (r2 < 0.f));
      pg.gd = md * inv_d * (float)((rd > 0.f) - (rd < 0.f));
      lpix = inv_c * (fabsf(r0) + fabsf(r1) + fabsf(r2)) + md * inv_d * fabsf(rd);
      if (color) {
        float* cb = color + 3 * c.vd.pix_off + off;
        cb[0] = s.C0;
        cb[hw] = s.C1;
        cb[2 * hw] = s.C2;
      }
      if (depth) depth[c.pix] = s.D;
      if (trans) trans[c.pix] = s.T;
    }
    if (loss_part) {
      // one plain store per (tile, quadrant); summed per view after the backward
      const float ws = wave_sum(lpix);
      if (lane == 0) loss_part[kWaves * tile + quad] = ws;
    }
    backward_walk<SM, true>(c, records, pairs, sigma, s.last, s.Tb, pg, srec, sface, sint, grad_acc, sig_acc,
                            persp_acc);
    if (!persistent) break;
  }
}

// ---------------------------------------------------------------------------- face backward
// Chain rule from the record parameters to the projected vertices (eq. 2-3 setup, in FP64),
// then through the pinhole projection to camera space, to world space (R^T) and to the
// se(3) pose (eq. 7: dv_C/dtau = [I, -[v_C]x]); vertex opacities get dL/do_F / 3 and
// vertex colours the barycentric weights' share.  One thread per face; loops over views.

__device__ __forceinline__ void load_pose_d(const float* __restrict__ poses, int v, double R[9], double t[3]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = (double)poses[12 * v + i];
#pragma unroll
  for (int i = 0; i < 3; ++i) t[i] = (double)poses[12 * v + 9 + i];
}

// Stage layout written into a consumed accumulator slot (floats): dL/dv_W for the three
// vertices [0..8] (vertex k, axis a at 3k + a), vertex colour gradients [9..17]
// (9 + 3k + ch), vertex opacity gradient [18] (the same for the three vertices).
constexpr int kStageFloats = 19;

__global__ __launch_bounds__(256) void k_face_bwd(tsr_scene_dev sc, const float* __restrict__ poses, ViewTable vt,
                                                  const uint32_t* __restrict__ vis_total,
                                                  const uint32_t* __restrict__ vis_dense,
                                                  const float* __restrict__ records, acc_t* grad_acc,
                                                  const float* __restrict__ persp_acc,
                                                  double* __restrict__ pose_acc, int want_vertices,
                                                  const float* __restrict__ loss_part, double* __restrict__ loss_acc) {
  const bool persp = persp_acc != nullptr;        // perspective-correct records
  __shared__ double s_pose[TSR_MAX_VIEWS * 6];    // this workgroup's pose sums, per view
  for (int k = threadIdx.x; k < TSR_MAX_VIEWS * 6; k += blockDim.x) s_pose[k] = 0.0;
  __syncthreads();
  if (loss_part) {
    // per-view loss: each thread adds one tile's four quadrant parts; waves whose tiles all
    // belong to one view (all but at most one wave per view boundary) add one FP64 atomic
    const int lane = threadIdx.x & 63;
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < vt.n_tiles; t0 += (int64_t)gridDim.x * blockDim.x) {
      const int64_t t = t0 + threadIdx.x;
      double x = 0.0;
      int v = -1;
      if (t < vt.n_tiles) {
        const float4 q = reinterpret_cast<const float4*>(loss_part)[t];
        x = ((double)q.x + (double)q.y) + ((double)q.z + (double)q.w);
        v = view_of_tile(vt, (int)t);
      }
      const int v0 = __shfl(v, 0, 64);
      double* lc = loss_acc + (int64_t)(blockIdx.x % kSumCopies) * vt.n_views;
      if (__ballot(v == v0 || v < 0) == ~0ull) {
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0 && v0 >= 0) unsafeAtomicAdd(&lc[v0], x);
      } else if (v >= 0) {
        unsafeAtomicAdd(&lc[v], x);
      }
    }
  }
  const int64_t M = vt.n_faces;
  const int64_t N = sc.n_vertices;
  const int64_t nf = (int64_t)vt.n_views * M;
  const int64_t total = min((int64_t)*vis_total, nf);
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < total; i0 += (int64_t)gridDim.x * blockDim.x) {
  const int64_t i = i0 + threadIdx.x;
  double pose6[6] = {0, 0, 0, 0, 0, 0};
  int v = -1;
  int64_t g = -1;
  if (i < total) {
    g = (int64_t)vis_dense[i];
    if (g >= nf) g = -1;                                            // never from a valid binning
  }
  if (g >= 0) {
    v = (int)(g / M);
    const int64_t m = g - (int64_t)v * M;
    int64_t vid[3];
    if (sc.faces) {
      for (int k = 0; k < 3; ++k) vid[k] = (int64_t)sc.faces[3 * m + k];
    } else {
      for (int k = 0; k < 3; ++k) vid[k] = 3 * m + k;
    }
    double gW[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // dL/dv_W per vertex
    double gcolv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // dL/dc per vertex, channel
    acc_t A[kGradDwords];                                  // read the whole slot before reusing it
#pragma unroll
    for (int k = 0; k < kGradDwords; ++k) A[k] = grad_acc[g * kGradDwords + k];
    const float* rec = records + g * kRecDwords;
    const ViewDesc vd = vt.v[v];
    double R[9], t[3];
    load_pose_d(poses, v, R, t);
    double vc[3][3], q[3][2];
    for (int k = 0; k < 3; ++k) {
      const double w0 = (double)sc.pos[vid[k]], w1 = (double)sc.pos[N + vid[k]], w2 = (double)sc.pos[2 * N + vid[k]];
      for (int a = 0; a < 3; ++a) vc[k][a] = R[3 * a] * w0 + R[3 * a + 1] * w1 + R[3 * a + 2] * w2 + t[a];
      q[k][0] = (double)vd.fx * vc[k][0] / vc[k][2] + (double)vd.cx;
      q[k][1] = (double)vd.fy * vc[k][1] / vc[k][2] + (double)vd.cy;
    }
    // ---- forward quantities of the setup
    const double a2 = (q[1][0] - q[0][0]) * (q[2][1] - q[0][1]) - (q[1][1] - q[0][1]) * (q[2][0] - q[0][0]);
    const double so = a2 >= 0.0 ? 1.0 : -1.0;
    const double area = fabs(a2);
    double e[3][2], len[3], n[3][2], perim = 0.0;
    for (int k = 0; k < 3; ++k) {
      const int k1 = (k + 1) % 3;
      e[k][0] = q[k1][0] - q[k][0];
      e[k][1] = q[k1][1] - q[k][1];
      len[k] = sqrt(e[k][0] * e[k][0] + e[k][1] * e[k][1]);
      perim += len[k];
    }
    // reciprocals once: the chain rule below multiplies (its results are compared within a
    // relative tolerance, not bit for bit)
    const double inv_perim = 1.0 / perim;
    const double r = area * inv_perim;
    const double inv_r = 1.0 / r;
    double inv_len[3];
    for (int k = 0; k < 3; ++k) inv_len[k] = 1.0 / len[k];
    for (int k = 0; k < 3; ++k) {
      n[k][0] = so * e[k][1] * inv_len[k];
      n[k][1] = -so * e[k][0] * inv_len[k];
    }
    const double U0 = (double)rec[kRecU0], V0 = (double)rec[kRecV0];
    double ca[3], cb[3], cc[3];       // edge coefficients a_k, b_k, c_k
    for (int k = 0; k < 3; ++k) {
      ca[k] = -n[k][0] * inv_r;
      cb[k] = -n[k][1] * inv_r;
      cc[k] = -(n[k][0] * (U0 - q[k][0]) + n[k][1] * (V0 - q[k][1])) * inv_r;
    }
    double colv[3][3];                // vertex colours [vertex][ch]
    for (int k = 0; k < 3; ++k)
      for (int ch = 0; ch < 3; ++ch) colv[k][ch] = (double)sc.col[ch * N + vid[k]];
    // ---- reverse: colour planes P_ch = sum_k beta_k,ch a_k (same for Q with b, R with c),
    //      beta_k,ch = len_k col[opp(k)][ch] / perim, times 1 / z_opp(k) in the perspective-correct
    //      mode, which also has the plane of W = sum_k beta_k (a_k, b_k, c_k), beta_k =
    //      len_k / (perim z_opp(k)); those 1 / z factors add dL/dz of the vertices (giz)
    double gA[3], gB[3], gCc[3], glen[3] = {0, 0, 0}, gperim = 0.0;
    double wz[3], giz[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) wz[k] = persp ? 1.0 / vc[(k + 2) % 3][2] : 1.0;
    for (int k = 0; k < 3; ++k) {
      gA[k] = (double)A[kGEdge + 3 * k];
      gB[k] = (double)A[kGEdge + 3 * k + 1];
      gCc[k] = (double)A[kGEdge + 3 * k + 2];
    }
    for (int k = 0; k < 3; ++k) {
      const int o = (k + 2) % 3;
      for (int ch = 0; ch < 3; ++ch) {
        const double GP = (double)A[kGCol + 3 * ch], GQ = (double)A[kGCol + 3 * ch + 1], GR = (double)A[kGCol + 3 * ch + 2];
        const double beta = len[k] * colv[o][ch] * inv_perim * wz[k];
        gA[k] += beta * GP;
        gB[k] += beta * GQ;
        gCc[k] += beta * GR;
        const double gbeta = GP * ca[k] + GQ * cb[k] + GR * cc[k];
        gcolv[o][ch] += gbeta * len[k] * inv_perim * wz[k];
        glen[k] += gbeta * colv[o][ch] * inv_perim * wz[k];
        gperim -= gbeta * beta * inv_perim;
        giz[k] += gbeta * len[k] * colv[o][ch] * inv_perim;
      }
    }
    if (persp) {
      const double GWa = (double)persp_acc[2 * g], GWb = (double)persp_acc[2 * g + 1], GWc = (double)A[kGWc];
      for (int k = 0; k < 3; ++k) {
        const double beta = len[k] * inv_perim * wz[k];
        gA[k] += beta * GWa;
        gB[k] += beta * GWb;
        gCc[k] += beta * GWc;
        const double gbeta = GWa * ca[k] + GWb * cb[k] + GWc * cc[k];
        glen[k] += gbeta * inv_perim * wz[k];
        gperim -= gbeta * beta * inv_perim;
        giz[k] += gbeta * len[k] * inv_perim;
      }
    }
    // ---- reverse: edge coefficients a = -n_x / r, b = -n_y / r, c = -n.(anchor - q_k) / r
    double gq[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    double gr = 0.0;
    double gn[3][2];
    for (int k = 0; k < 3; ++k) {
      gn[k][0] = -(gA[k] + gCc[k] * (U0 - q[k][0])) * inv_r;
      gn[k][1] = -(gB[k] + gCc[k] * (V0 - q[k][1])) * inv_r;
      gq[k][0] += gCc[k] * n[k][0] * inv_r;
      gq[k][1] += gCc[k] * n[k][1] * inv_r;
      gr -= (gA[k] * ca[k] + gB[k] * cb[k] + gCc[k] * cc[k]) * inv_r;
    }
    // ---- n_k = so (e_y, -e_x) / |e|
    double ge[3][2];
    for (int k = 0; k < 3; ++k) {
      const double dot = gn[k][0] * n[k][0] + gn[k][1] * n[k][1];
      const double gmx = (gn[k][0] - dot * n[k][0]) * inv_len[k];
      const double gmy = (gn[k][1] - dot * n[k][1]) * inv_len[k];
      ge[k][0] = -so * gmy;
      ge[k][1] = so * gmx;
    }
    // ---- r = area / perim; perim = sum len
    const double garea = gr * inv_perim;
    gperim += -gr * r * inv_perim;
    for (int k = 0; k < 3; ++k) {
      glen[k] += gperim;
      ge[k][0] += glen[k] * e[k][0] * inv_len[k];
      ge[k][1] += glen[k] * e[k][1] * inv_len[k];
    }
    // ---- area = so * a2, a2 = (q1 - q0) x (q2 - q0)
    const double ga2 = so * garea;
    gq[1][0] += ga2 * (q[2][1] - q[0][1]);
    gq[1][1] -= ga2 * (q[2][0] - q[0][0]);
    gq[2][0] -= ga2 * (q[1][1] - q[0][1]);
    gq[2][1] += ga2 * (q[1][0] - q[0][0]);
    gq[0][0] -= ga2 * ((q[2][1] - q[0][1]) - (q[1][1] - q[0][1]));
    gq[0][1] -= ga2 * ((q[1][0] - q[0][0]) - (q[2][0] - q[0][0]));
    // ---- e_k = q_{k+1} - q_k
    for (int k = 0; k < 3; ++k) {
      const int k1 = (k + 1) % 3;
      gq[k1][0] += ge[k][0];
      gq[k1][1] += ge[k][1];
      gq[k][0] -= ge[k][0];
      gq[k][1] -= ge[k][1];
    }
    // ---- projection and depth: q = (fx x / z + cx, fy y / z + cy), z_F = mean z (the
    //      perspective-correct mode has no z_F term; its 1 / z_k weights give -giz / z^2)
    const double gz3 = persp ? 0.0 : (double)A[kGZ] * (1.0 / 3.0);
    for (int k = 0; k < 3; ++k) {
      const double iz = 1.0 / vc[k][2];
      double gc[3];
      gc[0] = gq[k][0] * (double)vd.fx * iz;
      gc[1] = gq[k][1] * (double)vd.fy * iz;
      gc[2] = -(gq[k][0] * (double)vd.fx * vc[k][0] + gq[k][1] * (double)vd.fy * vc[k][1]) * iz * iz + gz3;
      if (persp) gc[2] -= giz[(k + 1) % 3] * iz * iz;      // vertex k faces edge (k + 1) % 3
      for (int a = 0; a < 3; ++a) gW[k][a] += R[a] * gc[0] + R[3 + a] * gc[1] + R[6 + a] * gc[2];
      pose6[0] += gc[0];
      pose6[1] += gc[1];
      pose6[2] += gc[2];
      pose6[3] += vc[k][1] * gc[2] - vc[k][2] * gc[1];
      pose6[4] += vc[k][2] * gc[0] - vc[k][0] * gc[2];
      pose6[5] += vc[k][0] * gc[1] - vc[k][1] * gc[0];
    }
    // dL/do_F to each vertex: a third for the mean; all of it, to one vertex, for the minimum
    const double gop = sc.opa_min ? (double)A[kGOpa] : (double)A[kGOpa] * (1.0 / 3.0);
    if (want_vertices) {
      float* stage = reinterpret_cast<float*>(grad_acc + g * kGradDwords);
      for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) {
          stage[3 * k + a] = (float)gW[k][a];
          stage[9 + 3 * k + a] = (float)gcolv[k][a];
        }
      stage[18] = (float)gop;
    }
  }
  // ---- pose gradient: a wave whose faces all belong to one view (always, for one view) adds
  //      its reduced sums, other waves each lane's, into the workgroup's per-view FP64 sums
  if (pose_acc) {
    const int lane = threadIdx.x & 63;
    const int v0 = __shfl(v, 0, 64);
    if (__ballot(v == v0 || v < 0) == ~0ull) {
      for (int c = 0; c < 6; ++c) {
        double x = v >= 0 ? pose6[c] : 0.0;
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0 && v0 >= 0) atomicAdd(&s_pose[v0 * 6 + c], x);
      }
    } else if (v >= 0) {
      for (int c = 0; c < 6; ++c) atomicAdd(&s_pose[v * 6 + c], pose6[c]);
    }
  }
  }
  // ---- one FP64 atomic per view and component into this workgroup's copy
  if (pose_acc) {
    __syncthreads();
    for (int k = threadIdx.x; k < 6 * vt.n_views; k += blockDim.x)
      if (s_pose[k] != 0.0) unsafeAtomicAdd(&pose_acc[(int64_t)(blockIdx.x % kSumCopies) * vt.n_views * 6 + k], s_pose[k]);
  }
}

// Float outputs of the FP64 pose and loss sums (adding their kSumCopies copies).
__device__ __forceinline__ void write_sums(const ViewTable& vt, const double* __restrict__ pose_acc,
                                           float* __restrict__ grad_pose, const double* __restrict__ loss_acc,
                                           float* __restrict__ loss) {
  const int nv = vt.n_views;
  for (int k = threadIdx.x; k < 7 * nv; k += blockDim.x) {
    const bool is_pose = k < 6 * nv;
    if (is_pose ? !grad_pose : !loss) continue;
    const double* src = is_pose ? pose_acc + k : loss_acc + (k - 6 * nv);
    const int stride = is_pose ? 6 * nv : nv;
    double t = 0.0;
#pragma unroll 8
    for (int c = 0; c < kSumCopies; ++c) t += src[(int64_t)c * stride];
    if (is_pose) grad_pose[k] = (float)t;
    else loss[k - 6 * nv] = (float)t;
  }
}

// Per-view L1 loss: FP64 sum of the (tile, quadrant) parts of the view's tiles, by one
// workgroup of kBlock threads (every thread calls).
__device__ void reduce_view_losses(const ViewTable& vt, const float* __restrict__ loss_part, float* __restrict__ loss) {
  __shared__ double red[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = 0; v < vt.n_views; ++v) {
    const int64_t p0 = (int64_t)kWaves * vt.v[v].tile_off;
    const int np = kWaves * vt.v[v].tiles_x * vt.v[v].tiles_y;
    double x = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) x += (double)loss_part[p0 + i];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kWaves; ++w) t += red[w];
      loss[v] = (float)t;
    }
    __syncthreads();
  }
}

// Per face: sum the staged vertex gradients over the views that see it and write them.
// Soups write every vertex once (zero for faces no view sees); indexed meshes add into
// zero-filled outputs.  Workgroup 0 also converts the FP64 pose and loss sums (complete once
// the face backward has finished) to the float outputs.
__global__ __launch_bounds__(256) void k_vertex_gather(tsr_scene_dev sc, ViewTable vt, const uint32_t* __restrict__ counts,
                                                       const acc_t* __restrict__ grad_acc,
                                                       const float* __restrict__ sig_acc, float* __restrict__ grad_pos,
                                                       float* __restrict__ grad_col, float* __restrict__ grad_opa,
                                                       const double* __restrict__ pose_acc, float* __restrict__ grad_pose,
                                                       const double* __restrict__ loss_acc, float* __restrict__ loss) {
  if (blockIdx.x == 0) write_sums(vt, pose_acc, grad_pose, loss_acc, loss);
  const int64_t M = vt.n_faces;
  const int64_t N = sc.n_vertices;
  const int64_t m0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t m = m0 + threadIdx.x;
  float acc[kStageFloats + 1];
#pragma unroll
  for (int k = 0; k <= kStageFloats; ++k) acc[k] = 0.f;
  bool any = false;
  float gsig = 0.f;     // dL/dsigma_m over the views (per-face exponents)
  if (m < M) {
    for (int v = 0; v < vt.n_views; ++v) {
      const int64_t g = (int64_t)v * M + m;
      if (counts[g] == 0) continue;
      any = true;
      if (sig_acc) gsig += sig_acc[g];
      static_assert(kGradDwords == 20 && sizeof(acc_t) >= 4, "a staged row starts with five 16-byte vectors");
      const float4* stage = reinterpret_cast<const float4*>(grad_acc + g * kGradDwords);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const float4 x = stage[q];
        acc[4 * q] += x.x;
        acc[4 * q + 1] += x.y;
        acc[4 * q + 2] += x.z;
        acc[4 * q + 3] += x.w;
      }
    }
  }
  if (sc.grad_face_sigma && m < M) sc.grad_face_sigma[m] = gsig;     // 0 for faces no view blends
  // with the minimum rule only the face's lowest-opacity vertex (lowest index on ties) gets the
  // opacity gradient
  int kmin = -1;
  if (sc.opa_min && m < M && any) {
    float om = 0.f;
    for (int k = 0; k < 3; ++k) {
      const int64_t vi = sc.faces ? (int64_t)sc.faces[3 * m + k] : 3 * m + k;
      const float o = sc.opa[vi];
      if (k == 0 || o < om) {
        om = o;
        kmin = k;
      }
    }
  }
  if (sc.faces) {
    if (m >= M || !any) return;
    for (int k = 0; k < 3; ++k) {
      const int64_t vi = (int64_t)sc.faces[3 * m + k];
      for (int a = 0; a < 3; ++a) {
        if (grad_pos) unsafeAtomicAdd(&grad_pos[a * N + vi], acc[3 * k + a]);
        if (grad_col) unsafeAtomicAdd(&grad_col[a * N + vi], acc[9 + 3 * k + a]);
      }
      if (grad_opa && (kmin < 0 || k == kmin)) unsafeAtomicAdd(&grad_opa[vi], acc[18]);
    }
    return;
  }
  // soup: the workgroup's 3 x 256 vertices are contiguous in each of the seven output arrays;
  // transpose through LDS so that every store instruction writes 256 contiguous bytes
  __shared__ float s_out[7][3 * 256];
  if (m < M) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        s_out[a][3 * threadIdx.x + k] = acc[3 * k + a];
        s_out[3 + a][3 * threadIdx.x + k] = acc[9 + 3 * k + a];
      }
      s_out[6][3 * threadIdx.x + k] = (kmin < 0 || k == kmin) ? acc[18] : 0.f;
    }
  }
  __syncthreads();
  const int nv = (int)(3 * min((int64_t)blockDim.x, M - m0));
  const int64_t v0 = 3 * m0;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (grad_pos) grad_pos[a * N + v0 + i] = s_out[a][i];
      if (grad_col) grad_col[a * N + v0 + i] = s_out[3 + a][i];
    }
    if (grad_opa) grad_opa[v0 + i] = s_out[6][i];
  }
}

// Set-up of a backward pass: zero the gradient accumulators of the visible (view, face) pairs
// (one 16-byte store per thread, grid-stride); workgroup 0 also zeroes the per-view FP64 pose
// and loss accumulators and the persistent kernel's queue counter, and builds the
// longest-first tile order when `order` is given (tile counts the binning leaves it to).
__global__ __launch_bounds__(256) void k_prep_bwd(ViewTable vt, const uint32_t* __restrict__ vis_total,
                                                  const uint32_t* __restrict__ vis_dense, acc_t* __restrict__ grad_acc,
                                                  float* __restrict__ sig_acc, float* __restrict__ persp_acc,
                                                  double* __restrict__ pose_acc, double* __restrict__ loss_acc,
                                                  int* __restrict__ queue) {
  constexpr int kVec = (int)(kGradDwords * sizeof(acc_t)) / 16;      // 16-byte stores per row
  const int64_t nf = (int64_t)vt.n_views * vt.n_faces;
  const int64_t n = min((int64_t)*vis_total, nf) * kVec;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = (int64_t)vis_dense[i / kVec];
    if (g < nf) {
      reinterpret_cast<float4*>(grad_acc + g * kGradDwords)[i % kVec] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (sig_acc && i % kVec == 0) sig_acc[g] = 0.f;
      if (persp_acc && i % kVec == 1) reinterpret_cast<float2*>(persp_acc)[g] = make_float2(0.f, 0.f);
    }
  }
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < kSumCopies * 6 * vt.n_views; k += blockDim.x) pose_acc[k] = 0.0;
    for (int k = threadIdx.x; k < kSumCopies * vt.n_views; k += blockDim.x) loss_acc[k] = 0.0;
    if (queue && threadIdx.x == 0) *queue = 0;
  }
}

// Longest-first tile order of a binning with more tiles than the binning orders itself: one
// workgroup of 1,024 threads (a quarter of the per-thread iterations of a 256-thread one).
__global__ __launch_bounds__(1024) void k_build_order(const uint32_t* __restrict__ ranges, int n_tiles,
                                                      int* __restrict__ order) {
  __shared__ uint32_t hist[kOrderBuckets];
  __shared__ unsigned long long wsum[16];
  build_tile_order(ranges, n_tiles, order, hist, wsum);
}

// The longest-first order of the binning held in `ws`: built with the binning up to
// kOrderInSortMax tiles, else here (enqueued on `st` before the kernels that read it).
// `built`: a launch since the binning (a forward on the same stream) already built it.
static const int* tile_order(const ViewTable& vt, const WsLayout& L, char* ws, hipStream_t st, bool built = false) {
  int* order = reinterpret_cast<int*>(ws + L.order);
  if (vt.n_tiles > kOrderInSortMax && !built)
    TSR_LAUNCH("tile_order", k_build_order, dim3(1), dim3(1024), 0, st,
               reinterpret_cast<const uint32_t*>(ws + L.ranges), vt.n_tiles, order);
  return order;
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.f;
}

// Float outputs of the pose and loss sums.  `loss_part` is given when the face backward did
// not run (no faces): the per-view losses are then summed here from the (tile, quadrant) parts.
__global__ __launch_bounds__(kBlock) void k_finalize(ViewTable vt, const double* __restrict__ pose_acc,
                                                     float* __restrict__ grad_pose, const double* __restrict__ loss_acc,
                                                     const float* __restrict__ loss_part, float* __restrict__ loss) {
  if (loss_part) {
    write_sums(vt, pose_acc, grad_pose, loss_acc, nullptr);
    if (loss) reduce_view_losses(vt, loss_part, loss);
  } else {
    write_sums(vt, pose_acc, grad_pose, loss_acc, loss);
  }
}

// Soups may hold more vertices than the 3 M of their faces: those vertices get zero gradients
// (the vertex gather writes the faces' vertices only).
__global__ void k_zero_soup_tail(float* __restrict__ gp, float* __restrict__ gc, float* __restrict__ go, int64_t N,
                                 int64_t v0) {
  const int64_t n = N - v0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (gp) gp[a * N + v0 + i] = 0.f;
      if (gc) gc[a * N + v0 + i] = 0.f;
    }
    if (go) go[v0 + i] = 0.f;
  }
}

// ---------------------------------------------------------------------------- pose arithmetic
// Exp of tau = (rho, theta) in se(3), applied on the left of (R, t) (eq. 6):
//   R' = dR R,  t' = dR t + J rho,
// dR = I + A K + B K^2 (Rodrigues), J = I + B K + C K^2 (the left Jacobian of SO(3)),
// K = [theta]x, a = |theta|, A = sin a / a, B = (1 - cos a) / a^2, C = (a - sin a) / a^3
// (two-term series below a = 1e-4, where the closed forms lose digits).
__device__ void se3_exp_left(const double rho[3], const double th[3], const double R[9], const double t[3],
                             double nR[9], double nt[3]) {
  const double a2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
  const double a = sqrt(a2);
  double A, B, Cc;
  if (a < 1e-4) {
    A = 1.0 - a2 / 6.0;
    B = 0.5 - a2 / 24.0;
    Cc = 1.0 / 6.0 - a2 / 120.0;
  } else {
    A = sin(a) / a;
    B = (1.0 - cos(a)) / a2;
    Cc = (a - sin(a)) / (a2 * a);
  }
  const double K[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
  double dR[9], Jm[9];
  for (int i = 0; i < 9; ++i) {
    const double I = (i % 4 == 0) ? 1.0 : 0.0;
    dR[i] = I + A * K[i] + B * K2[i];
    Jm[i] = I + B * K[i] + Cc * K2[i];
  }
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) nR[3 * i + j] = dR[3 * i] * R[j] + dR[3 * i + 1] * R[3 + j] + dR[3 * i + 2] * R[6 + j];
    nt[i] = dR[3 * i] * t[0] + dR[3 * i + 1] * t[1] + dR[3 * i + 2] * t[2] + Jm[3 * i] * rho[0] + Jm[3 * i + 1] * rho[1] +
            Jm[3 * i + 2] * rho[2];
  }
}

__device__ __forceinline__ void load_pose_f64(const float* __restrict__ pose, double R[9], double t[3]) {
  for (int i = 0; i < 9; ++i) R[i] = (double)pose[i];
  for (int i = 0; i < 3; ++i) t[i] = (double)pose[9 + i];
}

__device__ __forceinline__ void store_pose_f64(float* __restrict__ pose, const double R[9], const double t[3]) {
  for (int i = 0; i < 9; ++i) pose[i] = (float)R[i];
  for (int i = 0; i < 3; ++i) pose[9 + i] = (float)t[i];
}

// Tracking step: T <- Exp(delta) T with delta = -(lr_t g_rho, lr_r g_theta).
__global__ void k_pose_step(float* __restrict__ poses, const float* __restrict__ grad_pose, int n_views, float lr_t,
                            float lr_r) {
  const int v = threadIdx.x;
  if (v >= n_views) return;
  double rho[3], th[3], R[9], t[3], nR[9], nt[3];
  for (int i = 0; i < 3; ++i) {
    rho[i] = -(double)lr_t * (double)grad_pose[6 * v + i];
    th[i] = -(double)lr_r * (double)grad_pose[6 * v + 3 + i];
  }
  load_pose_f64(poses + 12 * v, R, t);
  se3_exp_left(rho, th, R, t, nR, nt);
  store_pose_f64(poses + 12 * v, nR, nt);
}

// Poses of Exp(tau_v) T_v for a perturbation tau [V][6] = (rho, theta).
__global__ void k_pose_compose(const float* __restrict__ tau, const float* __restrict__ poses, int n_views,
                               float* __restrict__ out) {
  const int v = threadIdx.x;
  if (v >= n_views) return;
  double rho[3], th[3], R[9], t[3], nR[9], nt[3];
  for (int i = 0; i < 3; ++i) {
    rho[i] = (double)tau[6 * v + i];
    th[i] = (double)tau[6 * v + 3 + i];
  }
  load_pose_f64(poses + 12 * v, R, t);
  se3_exp_left(rho, th, R, t, nR, nt);
  store_pose_f64(out + 12 * v, nR, nt);
}

// Gradient with respect to tau of a loss evaluated at Exp(tau) T, from its left-perturbation
// gradient g at Exp(tau) T: Exp(tau + d) = Exp(J_l(tau) d) Exp(tau) to first order, so
// dL/dtau = J_l(tau)^T g.  J_l(tau) = sum_n ad(tau)^n / (n+1)! with the se(3) adjoint
// ad(rho, theta) = [[theta]x, [rho]x; 0, [theta]x] (translation first); the series is summed
// in FP64 until its terms fall below 1e-17 of the running sum (at most 80 terms).
__global__ void k_pose_tau_grad(const float* __restrict__ tau, const float* __restrict__ grad_pose, int n_views,
                                float* __restrict__ grad_tau) {
  const int v = threadIdx.x;
  if (v >= n_views) return;
  double ad[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) ad[i][j] = 0.0;
  const double r0 = tau[6 * v], r1 = tau[6 * v + 1], r2 = tau[6 * v + 2];
  const double t0 = tau[6 * v + 3], t1 = tau[6 * v + 4], t2 = tau[6 * v + 5];
  for (int b = 0; b < 2; ++b) {          // [theta]x on the two diagonal blocks
    const int o = 3 * b;
    ad[o][o + 1] = -t2; ad[o][o + 2] = t1;
    ad[o + 1][o] = t2;  ad[o + 1][o + 2] = -t0;
    ad[o + 2][o] = -t1; ad[o + 2][o + 1] = t0;
  }
  ad[0][4] = -r2; ad[0][5] = r1;          // [rho]x in the upper right block
  ad[1][3] = r2;  ad[1][5] = -r0;
  ad[2][3] = -r1; ad[2][4] = r0;
  double term[6][6], J[6][6], nxt[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) term[i][j] = J[i][j] = (i == j) ? 1.0 : 0.0;
  for (int n = 1; n <= 80; ++n) {        // term = ad^n / (n+1)!
    double tmax = 0.0, jmax = 0.0;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double s = 0.0;
        for (int k = 0; k < 6; ++k) s += term[i][k] * ad[k][j];
        nxt[i][j] = s / (double)(n + 1);
      }
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        term[i][j] = nxt[i][j];
        J[i][j] += term[i][j];
        tmax = fmax(tmax, fabs(term[i][j]));
        jmax = fmax(jmax, fabs(J[i][j]));
      }
    if (tmax <= 1e-17 * jmax) break;
  }
  double g[6];
  for (int i = 0; i < 6; ++i) g[i] = (double)grad_pose[6 * v + i];   // (grad_tau may alias grad_pose)
  for (int j = 0; j < 6; ++j) {
    double s = 0.0;
    for (int i = 0; i < 6; ++i) s += J[i][j] * g[i];
    grad_tau[6 * v + j] = (float)s;
  }
}

// ---------------------------------------------------------------------------- launchers

static inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

static int sigma_mode(float s) { return s == 1.f ? 1 : (s == 0.5f ? 2 : (s == 2.f ? 3 : 0)); }

// Per-face exponents (mode 4) whenever the scene has them, else the global sigma's mode; plus
// 8 for perspective-correct interpolation.
static int sigma_mode(const ViewTable& vt, const tsr_params& p) {
  return (vt.face_sigma ? 4 : sigma_mode(p.sigma)) | (p.perspective ? 8 : 0);
}

// switch over the kernel modes built: exponent modes 0-4, perspective-correct with 0-3
#define TSR_MODE_SWITCH(mode, X)                                                                   \
  switch (mode) {                                                                                  \
    case 1: X(1); break; case 2: X(2); break; case 3: X(3); break; case 4: X(4); break;            \
    case 8: X(8); break; case 9: X(9); break; case 10: X(10); break; case 11: X(11); break;        \
    default: X(0); break;                                                                          \
  }
// The separate forward and backward walks with the normal channels.  A normal is constant
// over its face, so perspective-correct interpolation leaves it unchanged.
#define TSR_NORMAL_SWITCH(mode, X)                                                                 \
  switch (mode) {                                                                                  \
    case 17: X(17); break; case 18: X(18); break; case 19: X(19); break; case 20: X(20); break;    \
    case 24: X(24); break; case 25: X(25); break; case 26: X(26); break; case 27: X(27); break;    \
    default: X(16); break;                                                                         \
  }

static unsigned tile_grid(int n_tiles) { return 8u * (unsigned)((n_tiles + 7) / 8); }

// Staging of the separate forward and backward kernels: cooperative for several views (their
// records outgrow the caches, and one shared copy per tile is read instead of four), per wave
// for one (measured on an MI355X at 1200x680 with 1M faces: 8 views 0.32 -> 0.28 ms forward and
// 0.72 -> 0.70 ms backward cooperatively, one view 0.068 -> 0.074 ms forward).  Their spans are
// 128 faces (the fused kernel's 256 would cap them at five workgroups per CU by LDS; the 8-view
// mapping step took 1.98 ms with 256, 1.90 with 192 and 1.89 with 128).
static bool separate_coop(const ViewTable& vt) { return vt.n_views > 1; }

// Per-face screen statistics of binned views: the same front-to-back walk and blending
// decisions as the forward pass (one wave per 8x8 quadrant, per-wave staging).  Each pixel
// counts 1 for the coverage of the face with the largest blending weight alpha T along its
// ray (the first in depth order on ties), summed per wave before the atomics; a face blended
// at any pixel is marked visible (one store per wave and face visit, from the first lane that
// blends it).
template <int SM>
__global__ __launch_bounds__(kBlock) void k_face_stats(ViewTable vt, const float* __restrict__ records,
                                                       const uint64_t* __restrict__ pairs,
                                                       const uint32_t* __restrict__ ranges, float sigma, float t_min,
                                                       uint32_t* __restrict__ coverage, uint32_t* __restrict__ visible,
                                                       const int* __restrict__ order) {
  __shared__ float4 srec[kWaves][kBatch * 6];
  __shared__ uint32_t sface[kWaves][kBatch];
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int tile = tile_of_block_ordered(vt.n_tiles, order);
  if (tile < 0) return;
  TileCtx c;
  tile_ctx(vt, ranges, tile, wv, c);
  float T = c.inside ? 1.f : 0.f, best_w = 0.f;
  int best = -1;
  const float dxb = (float)c.px, dyb = (float)c.py;
  for (uint32_t b0 = c.start; b0 < c.end; b0 += kBatch) {
    if (ballot(live(T, t_min)) == 0) break;
    const int n = (int)min((uint32_t)kBatch, c.end - b0);
    stage_batch(records, pairs, b0, n, srec[wv], sface[wv]);
    unsigned long long mask = batch_hit_mask<SM>(srec[wv], n, c.bx, c.by);
    bool lv = live(T, t_min);
    while (mask) {
      const int j = __builtin_ctzll(mask);
      mask &= mask - 1;
      Rec rc;
      load_rec(srec[wv], j, rc);
      PixelEval e;
      const float dx = dxb - rc.f[kRecU0];
      const float dy = dyb - rc.f[kRecV0];
      const bool act = eval_face<SM>(rc, dx, dy, sigma, e) && lv;
      const float a = act ? e.alpha : 0.f;
      const float w = a * T;
      const uint32_t g = sface[wv][j];
      if (act && w > best_w) {
        best_w = w;
        best = (int)g;
      }
      const unsigned long long bm = ballot(act);
      if (visible && bm != 0ull && lane == __builtin_ctzll(bm)) visible[g] = 1u;
      T = T * (1.f - a);
      lv = live(T, t_min);
      if (ballot(lv) == 0) break;
    }
  }
  if (coverage) {
    // one atomic per distinct dominant face of the wave, adding its number of pixels (a large
    // face dominates many pixels, and atomics on one address serialise)
    bool pending = best >= 0;
    for (;;) {
      const unsigned long long pm = ballot(pending);
      if (pm == 0ull) break;
      const int leader = __builtin_ctzll(pm);
      const int f = __shfl(best, leader, 64);
      const unsigned long long same = ballot(pending && best == f);
      if (lane == leader) atomicAdd(&coverage[f], (uint32_t)__popcll(same));
      if (best == f) pending = false;
    }
  }
}

hipError_t launch_face_stats(const ViewTable& vt, const tsr_params& p, const WsLayout& L, char* ws,
                             uint32_t* coverage, uint32_t* visible, hipStream_t st) {
  const float* records = reinterpret_cast<const float*>(ws + L.records);
  const uint64_t* pairs = reinterpret_cast<const uint64_t*>(ws + L.pairs);
  const uint32_t* ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
  const int* border = tile_order(vt, L, ws, st);     // longest lists first
  const int64_t nf = (int64_t)vt.n_views * vt.n_faces;
  const unsigned fg = (unsigned)std::min<int64_t>((nf + 255) / 256, 4096);
  if (nf > 0) {
    if (coverage) TSR_LAUNCH("fill_stats", k_fill_f32, dim3(fg), dim3(256), 0, st, reinterpret_cast<float*>(coverage), nf);
    if (visible) TSR_LAUNCH("fill_stats", k_fill_f32, dim3(fg), dim3(256), 0, st, reinterpret_cast<float*>(visible), nf);
  }
  const dim3 grid(tile_grid(vt.n_tiles)), block(kBlock);
#define TSR_STATS(S) TSR_LAUNCH("face_stats", k_face_stats<S>, grid, block, 0, st, vt, records, pairs, ranges, p.sigma, p.t_min, coverage, visible, border)
  TSR_MODE_SWITCH(sigma_mode(vt, p), TSR_STATS)
#undef TSR_STATS
  return hipGetLastError();
}

hipError_t launch_forward(const ViewTable& vt, const tsr_params& p, const WsLayout& L, char* ws, float* color,
                          float* depth, float* trans, hipStream_t st, const NormalChannels* nc) {
  const float* records = reinterpret_cast<const float*>(ws + L.records);
  const uint64_t* pairs = reinterpret_cast<const uint64_t*>(ws + L.pairs);
  const uint32_t* ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
  const int* border = tile_order(vt, L, ws, st);     // longest lists first
  int* n_last = reinterpret_cast<int*>(ws + L.n_last);
  float* t_last = reinterpret_cast<float*>(ws + L.t_last);
  const dim3 grid(tile_grid(vt.n_tiles)), block(kBlock);
  NormalIn nin{};
  if (nc)
    nin = NormalIn{reinterpret_cast<const float4*>(nc->face_normal), nullptr, nc->map, nc->poses, nc->target,
                   nullptr, nc->part, nc->w_norm, vt.n_faces};
  const bool coop = separate_coop(vt);
#define TSR_FWD(S)                                                                                 \
  {                                                                                                \
    auto kf = coop ? k_blend_fwd<S, true> : k_blend_fwd<S, false>;                                 \
    TSR_LAUNCH("blend_fwd", kf, grid, block, 0, st, vt, records, pairs, ranges, p.sigma, p.t_min, color, depth, \
               trans, n_last, t_last, border, nin);                                                \
  }
  if (nc) {
    TSR_NORMAL_SWITCH(sigma_mode(vt, p) | 16, TSR_FWD)
  } else {
    TSR_MODE_SWITCH(sigma_mode(vt, p), TSR_FWD)
  }
#undef TSR_FWD
  return hipGetLastError();
}

hipError_t launch_backward(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                           const WsLayout& L, char* ws, const float* gcolor, const float* gdepth,
                           const float* gtrans, const float* tcolor, const float* tdepth, float* color,
                           float* depth, float* trans, float* loss, float* grad_pos, float* grad_col,
                           float* grad_opa, float* grad_pose, bool fused_train, const TrainSchedule& sched,
                           hipStream_t st, const NormalChannels* nc, bool order_built) {
  const uint32_t* vis_total = reinterpret_cast<const uint32_t*>(ws + L.vis_total);
  const uint32_t* vis_dense = reinterpret_cast<const uint32_t*>(ws + L.vis_dense);
  const uint32_t* counts = reinterpret_cast<const uint32_t*>(ws + L.counts);
  const float* records = reinterpret_cast<const float*>(ws + L.records);
  const uint64_t* pairs = reinterpret_cast<const uint64_t*>(ws + L.pairs);
  const uint32_t* ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
  const int* n_last = reinterpret_cast<const int*>(ws + L.n_last);
  const float* t_last = reinterpret_cast<const float*>(ws + L.t_last);
  acc_t* grad_acc = reinterpret_cast<acc_t*>(ws + L.grad_acc);
  double* pose_acc = reinterpret_cast<double*>(ws + L.pose_acc);
  float* sig_acc = vt.face_sigma ? reinterpret_cast<float*>(ws + L.sig_acc) : nullptr;
  float* persp_acc = p.perspective ? reinterpret_cast<float*>(ws + L.persp_acc) : nullptr;
  float* loss_part = reinterpret_cast<float*>(ws + L.loss_part);
  double* loss_acc = reinterpret_cast<double*>(ws + L.loss_acc);
  const int64_t nf = (int64_t)vt.n_views * vt.n_faces;
  const int* order = nullptr;
  int* queue = nullptr;
  // the separate backward always walks longest-first; the fused kernel when its schedule says so
  if (!fused_train || sched.order) order = tile_order(vt, L, ws, st, order_built);
  if (fused_train && sched.persistent) queue = reinterpret_cast<int*>(ws + L.hdr_queue);
  {
    const int64_t rows16 = nf * (int64_t)((kGradDwords * sizeof(acc_t)) / 16);
    const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(grid_for(rows16, 256), 1), 2048);
    TSR_LAUNCH("prep_bwd", k_prep_bwd, dim3(g), dim3(256), 0, st, vt, vis_total, vis_dense, grad_acc, sig_acc,
               persp_acc, pose_acc, loss_acc, queue);
  }
  const dim3 block(kBlock);
  const int sm = sigma_mode(vt, p);
  if (!fused_train) {
    const dim3 grid(tile_grid(vt.n_tiles));
    const int* border = order;
    NormalIn nin{};
    if (nc)
      nin = NormalIn{reinterpret_cast<const float4*>(nc->face_normal), reinterpret_cast<float4*>(nc->grad), nullptr,
                     nc->poses, nc->target, nc->count, nullptr, nc->w_norm, vt.n_faces};
    const bool coop = separate_coop(vt);
#define TSR_BWD(S)                                                                                 \
  {                                                                                                \
    auto kb = coop ? k_blend_bwd<S, true> : k_blend_bwd<S, false>;                                 \
    TSR_LAUNCH("blend_bwd", kb, grid, block, 0, st, vt, records, pairs, ranges, p.sigma, n_last, t_last, gcolor, \
               gdepth, gtrans, grad_acc, sig_acc, persp_acc, border, nin);                         \
  }
    if (nc) {
      TSR_NORMAL_SWITCH(sm | 16, TSR_BWD)
    } else {
      TSR_MODE_SWITCH(sm, TSR_BWD)
    }
#undef TSR_BWD
  } else {
    dim3 grid(tile_grid(vt.n_tiles));
    if (sched.order && !sched.persistent) grid = dim3(vt.n_tiles);
    if (sched.persistent) grid = dim3(sched.grid > 0 ? sched.grid : 2048);
#define TSR_TRAIN(S) TSR_LAUNCH("train_fused", k_train_fused<S>, grid, block, 0, st, vt, records, pairs, ranges, p.sigma, p.t_min, p.w_color, p.w_depth, tcolor, tdepth, color, depth, trans, loss ? loss_part : nullptr, grad_acc, sig_acc, persp_acc, order, queue, sched.persistent)
    TSR_MODE_SWITCH(sm, TSR_TRAIN)
#undef TSR_TRAIN
  }
  // per visible (view, face): chain rule and pose; then per face: vertex gradients summed
  // over the views (indexed meshes add into zero-filled outputs)
  const bool want_vertices = grad_pos || grad_col || grad_opa;
  const bool want_gather = want_vertices || sc.grad_face_sigma;
  const int64_t N = sc.n_vertices;
  if (sc.faces && want_vertices) {
    if (grad_pos) TSR_LAUNCH("zero_grads", k_fill_f32, dim3(2048), dim3(256), 0, st, grad_pos, 3 * N);
    if (grad_col) TSR_LAUNCH("zero_grads", k_fill_f32, dim3(2048), dim3(256), 0, st, grad_col, 3 * N);
    if (grad_opa) TSR_LAUNCH("zero_grads", k_fill_f32, dim3(2048), dim3(256), 0, st, grad_opa, N);
  }
  if (nf > 0) {
    const dim3 fgrid(std::min<unsigned>(grid_for(nf, 256), 2048u));
    TSR_LAUNCH("face_bwd", k_face_bwd, fgrid, dim3(256), 0, st, sc, poses, vt, vis_total, vis_dense, records,
               grad_acc, persp_acc, grad_pose ? pose_acc : nullptr, want_vertices ? 1 : 0, loss ? loss_part : nullptr,
               loss_acc);
    if (want_gather)
      TSR_LAUNCH("vertex_gather", k_vertex_gather, dim3(grid_for(vt.n_faces, 256)), dim3(256), 0, st, sc, vt, counts,
                 grad_acc, sig_acc, grad_pos, grad_col, grad_opa, pose_acc, grad_pose, loss_acc, loss);
    if (want_vertices && !sc.faces && N > 3 * vt.n_faces)
      TSR_LAUNCH("zero_grads", k_zero_soup_tail, dim3(std::min<unsigned>(grid_for(N - 3 * vt.n_faces, 256), 1024u)),
                 dim3(256), 0, st, grad_pos, grad_col, grad_opa, N, 3 * vt.n_faces);
  } else if (want_vertices && !sc.faces) {
    if (grad_pos) TSR_LAUNCH("zero_grads", k_fill_f32, dim3(2048), dim3(256), 0, st, grad_pos, 3 * N);
    if (grad_col) TSR_LAUNCH("zero_grads", k_fill_f32, dim3(2048), dim3(256), 0, st, grad_col, 3 * N);
    if (grad_opa) TSR_LAUNCH("zero_grads", k_fill_f32, dim3(2048), dim3(256), 0, st, grad_opa, N);
  }
  if ((nf <= 0 || !want_gather) && (grad_pose || loss))     // otherwise k_vertex_gather converts them
    TSR_LAUNCH("finalize", k_finalize, dim3(1), dim3(kBlock), 0, st, vt, pose_acc, grad_pose, loss_acc,
               nf <= 0 ? loss_part : nullptr, loss);
  return hipGetLastError();
}

hipError_t launch_pose_step(float* poses, const float* grad_pose, int n_views, float lr_t, float lr_r, hipStream_t st) {
  TSR_LAUNCH("pose_step", k_pose_step, dim3(1), dim3(64), 0, st, poses, grad_pose, n_views, lr_t, lr_r);
  return hipGetLastError();
}

hipError_t launch_pose_compose(const float* tau, const float* poses, int n_views, float* out, hipStream_t st) {
  TSR_LAUNCH("pose_compose", k_pose_compose, dim3(1), dim3(64), 0, st, tau, poses, n_views, out);
  return hipGetLastError();
}

hipError_t launch_pose_tau_grad(const float* tau, const float* grad_pose, int n_views, float* grad_tau, hipStream_t st) {
  TSR_LAUNCH("pose_tau_grad", k_pose_tau_grad, dim3(1), dim3(64), 0, st, tau, grad_pose, n_views, grad_tau);
  return hipGetLastError();
}

}  // namespace tsr
