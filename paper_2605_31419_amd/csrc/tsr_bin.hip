// Binning half of the hot path (gfx950): projection and per-face setup, tile counting,
// exclusive scan of tile counts, wave-cooperative key emission, per-tile depth sort.
//
// Projection (eq. 1), edge functions (eq. 2), inradius / incentre normalisation of the
// window (eq. 3), face opacity as the vertex mean and barycentric colour (Sec. 3.1) are
// evaluated once per (view, face) in FP64 and stored as an FP32 face-local record, so that
// the per-pixel work in the blend kernels is FP32 on small numbers.
#include "tsr_device.h"
#include "tsr_internal.h"

// The FP64 face setup decides integers (visibility, pixel rectangles, tight tile lists) that
// must equal a plain IEEE evaluation of the same formulas: no fused multiply-adds unless written.
#pragma clang fp contract(off)

namespace tsr {

// ---------------------------------------------------------------------------- face setup

struct FaceSetup {
  double vc[3][3];     // camera-space vertices
  double q[3][2];      // projected vertices
  double n[3][2];      // outward unit edge normals
  double len[3];       // edge lengths, edge k = q_k -> q_{k+1}
  double perim, area2, r, so;
  double zf;
  int u0, u1, v0, v1;  // pixel rectangle (inclusive), valid when visible
};

__device__ __forceinline__ void load_pose(const float* __restrict__ poses, int v, double R[9], double t[3]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = (double)poses[12 * v + i];
#pragma unroll
  for (int i = 0; i < 3; ++i) t[i] = (double)poses[12 * v + 9 + i];
}

__device__ __forceinline__ void face_vertices(const tsr_scene_dev& sc, int64_t m, int64_t vid[3]) {
  if (sc.faces) {
#pragma unroll
    for (int k = 0; k < 3; ++k) vid[k] = (int64_t)sc.faces[3 * m + k];
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) vid[k] = 3 * m + k;
  }
}

// Returns true when the face survives culling and overlaps the image.
__device__ bool setup_face(const tsr_scene_dev& sc, const int64_t vid[3], const double R[9], const double t[3],
                           const ViewDesc& vd, float z_near, float r_min, FaceSetup& f) {
  const int64_t N = sc.n_vertices;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double w0 = (double)sc.pos[vid[k]], w1 = (double)sc.pos[N + vid[k]], w2 = (double)sc.pos[2 * N + vid[k]];
#pragma unroll
    for (int a = 0; a < 3; ++a) f.vc[k][a] = R[3 * a] * w0 + R[3 * a + 1] * w1 + R[3 * a + 2] * w2 + t[a];
  }
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) ok = ok && (f.vc[k][2] >= (double)z_near);
  if (!ok) return false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f.q[k][0] = (double)vd.fx * f.vc[k][0] / f.vc[k][2] + (double)vd.cx;
    f.q[k][1] = (double)vd.fy * f.vc[k][1] / f.vc[k][2] + (double)vd.cy;
  }
  double a2 = (f.q[1][0] - f.q[0][0]) * (f.q[2][1] - f.q[0][1]) - (f.q[1][1] - f.q[0][1]) * (f.q[2][0] - f.q[0][0]);
  f.so = a2 >= 0.0 ? 1.0 : -1.0;
  f.area2 = fabs(a2);
  f.perim = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3;
    double ex = f.q[k1][0] - f.q[k][0], ey = f.q[k1][1] - f.q[k][1];
    f.len[k] = sqrt(ex * ex + ey * ey);
    f.perim += f.len[k];
  }
  f.r = f.area2 / f.perim;
  if (!(f.r >= (double)r_min)) return false;
  double umin = fmin(f.q[0][0], fmin(f.q[1][0], f.q[2][0]));
  double umax = fmax(f.q[0][0], fmax(f.q[1][0], f.q[2][0]));
  double vmin = fmin(f.q[0][1], fmin(f.q[1][1], f.q[2][1]));
  double vmax = fmax(f.q[0][1], fmax(f.q[1][1], f.q[2][1]));
  // pixel range [ceil(max(min,-1)), floor(min(max, W))] clipped to the image
  double lu = ceil(fmax(umin, -1.0)), hu = floor(fmin(umax, (double)vd.width));
  double lv = ceil(fmax(vmin, -1.0)), hv = floor(fmin(vmax, (double)vd.height));
  f.u0 = (int)fmax(lu, 0.0);
  f.u1 = (int)fmin(hu, (double)(vd.width - 1));
  f.v0 = (int)fmax(lv, 0.0);
  f.v1 = (int)fmin(hv, (double)(vd.height - 1));
  return f.u0 <= f.u1 && f.v0 <= f.v1;
}

// Outward unit edge normals and the depth key of a face that passed setup_face.
__device__ __forceinline__ void face_normals(FaceSetup& f) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3;
    double ex = f.q[k1][0] - f.q[k][0], ey = f.q[k1][1] - f.q[k][1];
    f.n[k][0] = f.so * ey / f.len[k];
    f.n[k][1] = -f.so * ex / f.len[k];
  }
  f.zf = (f.vc[0][2] + f.vc[1][2] + f.vc[2][2]) / 3.0;   // exact division: it decides the depth order
}

// Edge lines L_k(p) = n_k . p + d_k of a face after face_normals (eq. 2, d_k = -n_k . q_k).
struct EdgeLines {
  double n[3][2], d[3];
  int u0, u1, v0, v1;    // the face's pixel rectangle
};

__device__ __forceinline__ void edge_lines(const FaceSetup& f, EdgeLines& e) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    e.n[k][0] = f.n[k][0];
    e.n[k][1] = f.n[k][1];
    e.d[k] = -(f.n[k][0] * f.q[k][0] + f.n[k][1] * f.q[k][1]);
  }
  e.u0 = f.u0; e.u1 = f.u1; e.v0 = f.v0; e.v1 = f.v1;
}

// Tight triangle-tile test: can view-local tile (x, y) hold a pixel the face covers?  A
// covered pixel has every L_k < 0, and an affine L_k is smallest over the tile's box of pixel
// centres (clipped to the face's rectangle) at one corner: the tile is kept when that smallest
// value is below 0 for all three edges.
__device__ __forceinline__ bool tile_may_cover(const EdgeLines& e, int x, int y) {
  const double ulo = fmax(16.0 * x, (double)e.u0), uhi = fmin(16.0 * x + 15.0, (double)e.u1);
  const double vlo = fmax(16.0 * y, (double)e.v0), vhi = fmin(16.0 * y + 15.0, (double)e.v1);
  bool keep = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u = e.n[k][0] > 0 ? ulo : uhi, v = e.n[k][1] > 0 ? vlo : vhi;
    const double lmin = e.n[k][0] * u + e.n[k][1] * v + e.d[k];
    keep = keep && (lmin < 0);
  }
  return keep;
}

// The owner lane's edge lines, read by the other lanes of the wave.
__device__ __forceinline__ void shfl_lines(const EdgeLines& e, int owner, EdgeLines& o) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    o.n[k][0] = __shfl(e.n[k][0], owner, 64);
    o.n[k][1] = __shfl(e.n[k][1], owner, 64);
    o.d[k] = __shfl(e.d[k], owner, 64);
  }
  o.u0 = __shfl(e.u0, owner, 64);
  o.u1 = __shfl(e.u1, owner, 64);
  o.v0 = __shfl(e.v0, owner, 64);
  o.v1 = __shfl(e.v1, owner, 64);
}

// Vertex colours [channel][vertex] and opacities of a face (loaded before its setup so that
// their latency overlaps the FP64 work).
struct FaceAttr {
  float col[3][3];
  float opa[3];
  int opa_min;     // face opacity = min of the vertex opacities instead of their mean
  float sigma;     // window exponent of the face (eq. 3)
  int persp;       // perspective-correct interpolation: numerator and denominator planes
};

__device__ __forceinline__ void load_attr(const tsr_scene_dev& sc, int64_t m, const int64_t vid[3], float sigma,
                                          int persp, FaceAttr& a) {
  const int64_t N = sc.n_vertices;
  a.sigma = sc.face_sigma ? sc.face_sigma[m] : sigma;
  a.persp = persp;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) a.col[ch][k] = sc.col[ch * N + vid[k]];
    a.opa[k] = sc.opa[vid[k]];
  }
  a.opa_min = sc.opa_min;
}

// Writes the FP32 face-local record of a visible face (after face_normals).
__device__ __forceinline__ void write_record(const FaceAttr& at, const FaceSetup& f, float* __restrict__ dst_rec) {
  float rec[kRecDwords];
  const double inv_r = 1.0 / f.r;
  double a[3], b[3], c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a[k] = -f.n[k][0] * inv_r;
    b[k] = -f.n[k][1] * inv_r;
    c[k] = -(f.n[k][0] * ((double)f.u0 - f.q[k][0]) + f.n[k][1] * ((double)f.v0 - f.q[k][1])) * inv_r;
    rec[kRecEdge + 3 * k] = (float)a[k];
    rec[kRecEdge + 3 * k + 1] = (float)b[k];
    rec[kRecEdge + 3 * k + 2] = (float)c[k];
  }
  const double inv_perim = 1.0 / f.perim;
  // lambda_opp(k) = E_k len_k / perimeter; opp(k) = (k + 2) % 3 is the vertex facing edge k.
  // Perspective-correct mode weights each vertex by 1 / z (its camera depth).
  double wz[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) wz[k] = at.persp ? 1.0 / f.vc[(k + 2) % 3][2] : 1.0;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    double P = 0, Q = 0, Rr = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double beta = f.len[k] * (double)at.col[ch][(k + 2) % 3] * inv_perim * wz[k];
      P += beta * a[k];
      Q += beta * b[k];
      Rr += beta * c[k];
    }
    rec[kRecCol + 3 * ch] = (float)P;
    rec[kRecCol + 3 * ch + 1] = (float)Q;
    rec[kRecCol + 3 * ch + 2] = (float)Rr;
  }
  rec[kRecOpa] = at.opa_min ? fminf(at.opa[0], fminf(at.opa[1], at.opa[2]))
                            : (float)(((double)at.opa[0] + (double)at.opa[1] + (double)at.opa[2]) / 3.0);
  rec[kRecZ] = (float)f.zf;
  rec[kRecU0] = (float)f.u0;          // exact: |u0| < 2^24
  rec[kRecV0] = (float)f.v0;
  rec[kRecU1V1] = __int_as_float(f.u1 | (f.v1 << 16));    // both below 2^14
  rec[kRecSigma] = at.sigma;
  if (at.persp) {
    // denominator plane W = sum_k lambda_opp(k) / z_opp(k) (1 / depth of the face's plane)
    double Wa = 0, Wb = 0, Wc = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double beta = f.len[k] * inv_perim * wz[k];
      Wa += beta * a[k];
      Wb += beta * b[k];
      Wc += beta * c[k];
    }
    rec[kRecWa] = (float)Wa;
    rec[kRecWb] = (float)Wb;
    rec[kRecWc] = (float)Wc;
  }
  float4* dst = reinterpret_cast<float4*>(dst_rec);
#pragma unroll
  for (int i = 0; i < kRecDwords / 4; ++i) dst[i] = make_float4(rec[4 * i], rec[4 * i + 1], rec[4 * i + 2], rec[4 * i + 3]);
}

// Conservative FP32 pre-test: true only when setup_face (FP64) is certain to cull the face,
// i.e. a vertex lies behind the near plane by more than the FP32 error bound, or the face's
// pixel range stays empty when every projected coordinate is widened by its error bound.
// Faces it does not reject go through setup_face; non-finite values are never rejected here.
// Error bounds: camera coordinates from three FMAs and an add of float inputs differ from the
// FP64 value by at most 4 ulp-units of sum |R_ai w_i| + |t_a| (bound used: 1e-6 x that sum);
// the projection adds the propagated coordinate error, the reciprocal (<= 1 ulp) and two
// roundings (bound used: 4x the first-order estimate, plus 1e-4 px).
// The world positions w[vertex][axis] are loaded by the caller (several faces' loads in flight).
__device__ __forceinline__ bool surely_culled(const float w[3][3], const float* __restrict__ pose, const ViewDesc& vd,
                                              float z_near) {
  float ulo = INFINITY, uhi = -INFINITY, vlo = INFINITY, vhi = -INFINITY;
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float w0 = w[k][0], w1 = w[k][1], w2 = w[k][2];
    float c[3], e[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float r0 = pose[3 * a], r1 = pose[3 * a + 1], r2 = pose[3 * a + 2], ta = pose[9 + a];
      c[a] = fmaf(r0, w0, fmaf(r1, w1, fmaf(r2, w2, ta)));
      e[a] = 1e-6f * (fabsf(r0 * w0) + fabsf(r1 * w1) + fabsf(r2 * w2) + fabsf(ta));
    }
    if (c[2] + e[2] < z_near) return true;           // FP64 depth below z_near as well
    const float zlo = c[2] - e[2];
    if (!(zlo > 0.f)) return false;                   // projection bound needs z > 0
    // hardware reciprocal (<= 1 ulp) times the coordinate: <= 1.5 ulp relative for q
    const float rz = __builtin_amdgcn_rcpf(c[2]), rzlo = __builtin_amdgcn_rcpf(zlo);
    const float qx = c[0] * rz, qy = c[1] * rz;
    const float dqx = (e[0] + fabsf(qx) * e[2]) * rzlo * 1.0001f + 3e-7f * fabsf(qx);
    const float dqy = (e[1] + fabsf(qy) * e[2]) * rzlo * 1.0001f + 3e-7f * fabsf(qy);
    const float u = fmaf(vd.fx, qx, vd.cx), v = fmaf(vd.fy, qy, vd.cy);
    const float du = 4.f * (fabsf(vd.fx) * dqx + 1.2e-7f * (fabsf(vd.fx * qx) + fabsf(vd.cx) + fabsf(u))) + 1e-4f;
    const float dv = 4.f * (fabsf(vd.fy) * dqy + 1.2e-7f * (fabsf(vd.fy * qy) + fabsf(vd.cy) + fabsf(v))) + 1e-4f;
    finite = finite && isfinite(u) && isfinite(v) && isfinite(du) && isfinite(dv);
    ulo = fminf(ulo, u - du);
    uhi = fmaxf(uhi, u + du);
    vlo = fminf(vlo, v - dv);
    vhi = fmaxf(vhi, v + dv);
  }
  if (!finite) return false;
  const float cu0 = fmaxf(ceilf(ulo), 0.f), cu1 = fminf(floorf(uhi), (float)(vd.width - 1));
  const float cv0 = fmaxf(ceilf(vlo), 0.f), cv1 = fminf(floorf(vhi), (float)(vd.height - 1));
  return cu0 > cu1 || cv0 > cv1;
}

// ---------------------------------------------------------------------------- wave expansion
// Spreads per-lane work lists (lane l owns cnt_l items) evenly over the 64 lanes: a wave
// prefix scan of the counts, then each lane finds the owner of its item by binary search
// over the inclusive prefix (held in lanes, read with ds_bpermute).  All lanes must be
// active.  fn(owner_lane, item_index_within_owner) runs once per item.
template <class F>
__device__ __forceinline__ void wave_expand(int cnt, F&& fn) {
  const int lane = threadIdx.x & 63;
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const int total = __shfl(incl, 63, 64);
  for (int base = 0; base < total; base += 64) {
    const int j = base + lane;
    int lo = 0, hi = 63;
#pragma unroll
    for (int s = 0; s < 6; ++s) {               // smallest lane with incl > j
      int mid = (lo + hi) >> 1;
      int im = __shfl(incl, mid, 64);
      if (im > j) hi = mid; else lo = mid + 1;
    }
    const int owner = lo;
    const int excl_owner = __shfl(incl, owner, 64) - __shfl(cnt, owner, 64);
    fn(j < total, owner, j - excl_owner);
  }
}

// wave_expand for item functions that return whether they kept their item: returns, on each
// lane, how many of its own items were kept (a ballot per round, masked to the lane's items).
template <class F>
__device__ __forceinline__ int wave_expand_count(int cnt, F&& fn) {
  const int lane = threadIdx.x & 63;
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const int total = __shfl(incl, 63, 64);
  int kept = 0;
  for (int base = 0; base < total; base += 64) {
    const int j = base + lane;
    int lo = 0, hi = 63;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      int mid = (lo + hi) >> 1;
      int im = __shfl(incl, mid, 64);
      if (im > j) hi = mid; else lo = mid + 1;
    }
    const int owner = lo;
    const int excl_owner = __shfl(incl, owner, 64) - __shfl(cnt, owner, 64);
    const bool k = fn(j < total, owner, j - excl_owner);
    const unsigned long long b = __ballot(k && j < total);
    // this lane's items in the round: positions [incl - cnt, incl) relative to base
    const int a = max(incl - cnt - base, 0), e = min(incl - base, 64);
    if (e > a) {
      const unsigned long long hi_mask = e == 64 ? ~0ull : ((1ull << e) - 1ull);
      kept += __popcll(b & hi_mask & ~((1ull << a) - 1ull));
    }
  }
  return kept;
}

// ---------------------------------------------------------------------------- kernels

// Projection workgroups of 256 threads, each taking ROUNDS x 256 consecutive (view, face)
// pairs, numbered face-major (the views of a face in adjacent lanes); per-(view, face) arrays
// are indexed by g = v * M + m (below 2^31: the entry points refuse larger V * M).  Two stages:
// the FP32 pre-test rejects the pairs that are certainly culled (the positions of all rounds
// are loaded before any test, so that their loads overlap); the remaining candidates are
// compacted in pair order into LDS and taken 256 at a time by the exact FP64 setup (the
// visibility decision, the pixel rectangle and, for visible faces, the record), one candidate
// per lane.  One round for a single view: its 3,900 workgroups of one partly used FP64 wave
// each overlap well, and workgroup b compacts its visible pairs (wave ballots, per-wave counts
// in LDS) into visible-list segment b.  Four rounds for several views (face-major, a workgroup
// of one round holds 256 / V faces): the FP64 waves are then full and the workgroups four times
// fewer (8 views of 1200x680 with 1M faces: 244 -> 190 us; one view 39 -> 44 us), and wave w of
// workgroup b appends its visible pairs of every chunk (at most 4 x 64) to segment 4 b + w, so
// the four segments stay balanced for the emission (one segment per chunk doubled the
// emission's time) and the compaction needs no barrier.  The dense visible list then follows
// the segments, not pair order (the face backward's gathers lose a little locality: +6 us).
// Four workgroups per CU: the FP64 setup then fits its registers without spilling (six
// spilled 28 registers to scratch and took 57 us against 48 us at 1200x680 with 1M faces).
template <bool TIGHT, int ROUNDS>
__global__ __launch_bounds__(256, 4) void k_project(tsr_scene_dev sc, const float* __restrict__ poses, ViewTable vt,
                                                 float z_near, float r_min, float sigma, int persp,
                                                 uint32_t* __restrict__ counts,
                                                 float* __restrict__ records, uint32_t* __restrict__ tile_cnt,
                                                 uint32_t* __restrict__ vis_cnt, VisEntry* __restrict__ vis_list) {
  static_assert(kProjBlock == 256, "four waves per projection workgroup: s_wave, s_cnt and the chunk size");
  constexpr int kPairs = ROUNDS * kProjBlock;
  __shared__ uint32_t s_wave[4];
  __shared__ uint32_t s_cnt[ROUNDS][4];
  __shared__ uint32_t s_cand[kPairs];
  const uint32_t M = (uint32_t)vt.n_faces, V = (uint32_t)vt.n_views, NF = V * M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t first = blockIdx.x * (uint32_t)kPairs;
  uint32_t ncand = 0u;
  {
    float w[ROUNDS][3][3];
    uint32_t gr[ROUNDS];
    int vr[ROUNDS];
    const int64_t N = sc.n_vertices;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      const uint32_t idx = first + (uint32_t)(r * kProjBlock) + threadIdx.x;
      const uint32_t id = idx < NF ? idx : 0u;        // lanes past the end test pair 0 and drop it
      const uint32_t m = id / V;
      vr[r] = (int)(id - m * V);
      gr[r] = (uint32_t)vr[r] * M + m;
      int64_t vid[3];
      face_vertices(sc, (int64_t)m, vid);
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) w[r][k][a] = sc.pos[a * N + vid[k]];
    }
    unsigned long long mask[ROUNDS];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      const bool in = first + (uint32_t)(r * kProjBlock) + threadIdx.x < NF;
      const bool cand = in && !surely_culled(w[r], poses + 12 * vr[r], vt.v[vr[r]], z_near);
      if (in && !cand) counts[gr[r]] = 0u;
      mask[r] = __ballot(cand);
      if (lane == 0) s_cnt[r][wave] = (uint32_t)__popcll(mask[r]);
    }
    __syncthreads();
    // candidates in pair order: round, then wave, then lane
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      uint32_t off = ncand + (uint32_t)__popcll(mask[r] & below);
      for (int q = 0; q < 4; ++q) {
        if (q < wave) off += s_cnt[r][q];
        ncand += s_cnt[r][q];
      }
      if ((mask[r] >> lane) & 1ull) s_cand[off] = gr[r];
    }
  }
  const int seg0 = (int)blockIdx.x * ROUNDS;
  const int nchunk = (int)((ncand + kProjBlock - 1u) / kProjBlock);
  if constexpr (ROUNDS == 1)
    if (nchunk == 0 && threadIdx.x == 0) vis_cnt[seg0] = 0u;
  __syncthreads();                                // s_cand complete
  uint32_t wcount = 0u;                           // several rounds: this wave's visible pairs so far
  // Chunk c of the candidates; false for a wave that has left (in the last chunk, whole waves
  // without a candidate leave at once, so their slots go to other workgroups during the FP64
  // stage; the barriers below then wait for the remaining waves only).
  auto chunk = [&](int c) -> bool {
    const uint32_t left = ncand - (uint32_t)(c * kProjBlock);
    // One round: candidate 64 w' + lane, w' the wave counted from wave b mod 4 of workgroup b,
    // so that the FP64 waves of neighbouring workgroups do not all sit on the same SIMD
    // (44.0 -> 42.5 us).  Several: the chunk's candidates round-robin over the waves
    // (c * 256 + 4 lane + wave), so that the views of one face, adjacent in pair order, land in
    // different waves' segments and the emission's expansion of larger faces is spread evenly
    // (8 views: emission 101 -> 69 us; with a contiguous quarter of the chunk per wave 84 us).
    const int wr = ROUNDS == 1 ? ((wave - (int)(blockIdx.x & 3u)) & 3) : wave;
    const int slot = ROUNDS == 1 ? wr * kWave + lane : lane * 4 + wave;
    const int nact = ROUNDS == 1 ? (left >= (uint32_t)kProjBlock ? 4 : (int)((left + 63u) >> 6))
                                 : (left >= 4u ? 4 : (int)left);
    if (wr >= nact) return false;
    // ---- exact setup of the chunk's candidates, one per lane
    int ntiles = 0, tx0 = 0, ty0 = 0, tw = 1, th = 1, tile_base = 0, tiles_x = 1;
    uint32_t zbits = 0u;
    uint32_t keep = 0xfu;        // tight binning: which tiles of a face over at most kSmallTiles are listed
    EdgeLines el{};              // tight binning: the face's edge lines (read by the larger faces' items)
    uint32_t g = 0u;
    if ((uint32_t)slot < left) {
      g = s_cand[c * kProjBlock + slot];
      const uint32_t v = g / M;
      const ViewDesc& vd = vt.v[v];
      double R[9], t[3];
      load_pose(poses, (int)v, R, t);
      int64_t vid[3];
      const int64_t m = (int64_t)(g - v * M);
      face_vertices(sc, m, vid);
      FaceAttr at;
      load_attr(sc, m, vid, sigma, persp, at);
      FaceSetup f;
      if (setup_face(sc, vid, R, t, vd, z_near, r_min, f)) {
        tx0 = f.u0 >> 4;
        ty0 = f.v0 >> 4;
        tw = (f.u1 >> 4) - tx0 + 1;
        th = (f.v1 >> 4) - ty0 + 1;
        ntiles = tw * th;
        tile_base = vd.tile_off;
        tiles_x = vd.tiles_x;
        face_normals(f);
        write_record(at, f, records + (int64_t)g * kRecDwords);
        zbits = __float_as_uint((float)f.zf);     // the record's z_F (set by face_normals)
        if constexpr (TIGHT) {
          edge_lines(f, el);
          if (ntiles <= kSmallTiles) {
            keep = 0u;
#pragma unroll
            for (int i = 0; i < kSmallTiles; ++i)
              if (i < ntiles && tile_may_cover(el, tx0 + i % tw, ty0 + i / tw)) keep |= 1u << i;
          }
        }
      }
      // listed tiles (larger faces under tight binning: corrected after their items are decided)
      counts[g] = ntiles <= kSmallTiles ? (uint32_t)__popc(keep & ((1u << ntiles) - 1u)) : (uint32_t)ntiles;
    }
    if constexpr (TIGHT) {
      if (ntiles > 0 && ntiles <= kSmallTiles && (keep & ((1u << ntiles) - 1u)) == 0u) ntiles = 0;   // no tile left
    }
    // ---- visible (view, face) pairs into the visible list, in candidate order: the workgroup's
    //      segment (one round) or the wave's own (several); wave ballots, no atomics
    const bool vis = ntiles > 0;
    uint4* ent = nullptr;
    {
      const unsigned long long vmask = __ballot(vis);
      uint32_t off = (uint32_t)__popcll(vmask & below);
      int seg = seg0;
      if constexpr (ROUNDS == 1) {
        if (lane == 0) s_wave[wr] = (uint32_t)__popcll(vmask);
        __syncthreads();
        for (int q = 0; q < wr; ++q) off += s_wave[q];
        if (wr == 0 && lane == 0) {
          uint32_t nvis = 0u;
          for (int q = 0; q < nact; ++q) nvis += s_wave[q];
          vis_cnt[seg] = nvis;
        }
      } else {
        seg = seg0 + wave;
        off += wcount;
        wcount += (uint32_t)__popcll(vmask);
      }
      ent = reinterpret_cast<uint4*>(vis_list + (int64_t)seg * kProjBlock + off);
      if (vis)
        ent[0] = make_uint4(g, (uint32_t)(tile_base + ty0 * tiles_x + tx0),
                            (uint32_t)(tw - 1) | ((uint32_t)(th - 1) << 10) | ((uint32_t)(tiles_x - 1) << 20), zbits);
    }
    // ---- per-tile counts.  A face overlapping at most kSmallTiles tiles takes its slot in each
    //      tile from the returning atomic and records it, so emission needs no atomics for it;
    //      larger faces are counted separately and spread over the wave.
    if (vis && ntiles <= kSmallTiles) {
      uint32_t sl[kSmallTiles];
#pragma unroll
      for (int i = 0; i < kSmallTiles; ++i)
        sl[i] = (i < ntiles && ((keep >> i) & 1u))
                    ? atomicAdd(&tile_cnt[kTileCntStride * (tile_base + (ty0 + i / tw) * tiles_x + tx0 + i % tw)], 1u)
                    : kSkipSlot;
      ent[1] = make_uint4(sl[0], sl[1], sl[2], sl[3]);
    }
    const int big = ntiles > kSmallTiles ? ntiles : 0;
    if (wave_max_int(big) == 0) return true;
    if constexpr (!TIGHT) {
      wave_expand(big, [&](bool valid, int owner, int i) {
        const int otx0 = __shfl(tx0, owner, 64), oty0 = __shfl(ty0, owner, 64), otw = __shfl(tw, owner, 64);
        const int obase = __shfl(tile_base, owner, 64), otx = __shfl(tiles_x, owner, 64);
        if (valid) atomicAdd(&tile_cnt[kTileCntStride * (obase + (oty0 + i / otw) * otx + otx0 + i % otw) + 2], 1u);
      });
    } else {
      const int kept = wave_expand_count(big, [&](bool valid, int owner, int i) {
        const int otx0 = __shfl(tx0, owner, 64), oty0 = __shfl(ty0, owner, 64), otw = __shfl(tw, owner, 64);
        const int obase = __shfl(tile_base, owner, 64), otx = __shfl(tiles_x, owner, 64);
        EdgeLines oe;
        shfl_lines(el, owner, oe);
        const int x = otx0 + i % otw, y = oty0 + i / otw;
        const bool k = valid && tile_may_cover(oe, x, y);
        if (k) atomicAdd(&tile_cnt[kTileCntStride * (obase + y * otx + x) + 2], 1u);
        return k;
      });
      if (big > 0) counts[g] = (uint32_t)kept;
    }
    return true;
  };
  if constexpr (ROUNDS == 1) {
    if (nchunk > 0) chunk(0);                    // straight-line: no loop for the compiler to hoist into
  } else {
    static_assert(ROUNDS * kWave <= kProjBlock, "a wave's visible pairs of every chunk fit its segment");
    for (int c = 0; c < nchunk; ++c)
      if (!chunk(c)) break;
    if (lane == 0) vis_cnt[seg0 + wave] = wcount;
  }
}

// Two workgroups of 1024 threads, working independently: (0) exclusive scan of the
// visible-face counts of the visible-list segments (offsets of the segments in the dense
// visible list); (1) exclusive scan of the tile counts into ranges, pair total K, overflow check against the capacity (all
// ranges empty on overflow), the small-face counts left in tile_cnt2 as the base of the
// larger faces' emission cursors, and the list of tiles too long for the one-wave sort.  Both
// scans run in rounds of kScanRound entries, each thread taking kScanPer consecutive ones (10:
// with 12 the 128 registers of a 1024-thread workgroup spill).
constexpr int kScanPer = 10;
constexpr int kScanRound = 1024 * kScanPer;

__global__ __launch_bounds__(1024) void k_scan_tiles(uint32_t* __restrict__ tile_cnt, uint32_t* __restrict__ ranges,
                                                     int n_tiles, int64_t capacity, int64_t* __restrict__ K_out,
                                                     uint32_t* __restrict__ overflow, const uint32_t* __restrict__ vis_cnt,
                                                     uint32_t* __restrict__ vis_off, uint32_t* __restrict__ vis_total,
                                                     int n_segments, uint32_t* __restrict__ long_cnt,
                                                     uint32_t* __restrict__ long_list) {
  // Loads and stores of a round are coalesced (entry base + 1024 k + tid); the entries reach
  // their owners (kScanPer consecutive ones each) and the results come back through s_x.  The
  // next round's loads are issued before the current round is scanned.
  __shared__ unsigned long long wsum[16];
  __shared__ uint2 s_x[kScanRound];
  const int tid = threadIdx.x;
  unsigned long long carry = 0, tot;
  if (blockIdx.x == 0) {
    // workgroup 0: offsets of the visible segments
    uint32_t ld[kScanPer], c[kScanPer];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int i = 1024 * k + tid;
      ld[k] = i < n_segments ? vis_cnt[i] : 0u;
    }
    for (int base = 0; base < n_segments; base += kScanRound) {
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) s_x[1024 * k + tid].x = ld[k];
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) {
        const int i = base + kScanRound + 1024 * k + tid;
        ld[k] = i < n_segments ? vis_cnt[i] : 0u;
      }
      __syncthreads();
      unsigned long long sum = 0;
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) {
        c[k] = s_x[tid * kScanPer + k].x;
        sum += c[k];
      }
      unsigned long long run = carry + block_excl_scan_u64(sum, wsum, &tot);   // (orders the reads above)
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) {
        s_x[tid * kScanPer + k].x = (uint32_t)run;
        run += c[k];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) {
        const int i = base + 1024 * k + tid;
        if (i < n_segments) vis_off[i] = s_x[1024 * k + tid].x;
      }
      carry += tot;
      __syncthreads();                 // s_x is refilled by the next round
    }
    if (tid == 0) *vis_total = (uint32_t)carry;
    return;
  }

  // workgroup 1: tile ranges; tiles longer than the one-wave sort takes are appended to the
  // long list (few; their order does not matter)
  uint32_t cs[kScanPer], cb[kScanPer];
  uint2 ld[kScanPer];                  // (small-face count, larger-face count) of an entry
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int i = 1024 * k + tid;
    ld[k] = i < n_tiles ? make_uint2(tile_cnt[kTileCntStride * i], tile_cnt[kTileCntStride * i + 2]) : make_uint2(0u, 0u);
  }
  uint2* ranges2 = reinterpret_cast<uint2*>(ranges);
  for (int base = 0; base < n_tiles; base += kScanRound) {
    const int i0 = base + tid * kScanPer;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s_x[1024 * k + tid] = ld[k];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int i = base + kScanRound + 1024 * k + tid;
      ld[k] = i < n_tiles ? make_uint2(tile_cnt[kTileCntStride * i], tile_cnt[kTileCntStride * i + 2])
                          : make_uint2(0u, 0u);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const uint2 c = s_x[tid * kScanPer + k];
      cs[k] = c.x;
      cb[k] = c.y;
    }
    // (the barriers inside the block scans below order these reads before the stores into s_x)
    unsigned long long sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) sum += (unsigned long long)cs[k] + cb[k];
    unsigned long long run = carry + block_excl_scan_u64(sum, wsum, &tot);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const unsigned long long c = (unsigned long long)cs[k] + cb[k];
      // start of the tile's range, and the base of its larger faces' cursor (after the
      // recorded slots)
      s_x[tid * kScanPer + k] = make_uint2((uint32_t)run, cs[k]);
      if (i0 + k < n_tiles && c > (unsigned long long)kWaveSortMax) long_list[atomicAdd(long_cnt, 1u)] = (uint32_t)(i0 + k);
      run += c;
    }
    __syncthreads();
    // a range ends where the next tile's starts; the round's last one at the round's total
    const uint32_t round_end = (uint32_t)(carry + tot);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int j = 1024 * k + tid, i = base + j;
      if (i < n_tiles) {
        const uint2 x = s_x[j];
        const uint32_t end = (j + 1 < kScanRound && i + 1 < n_tiles) ? s_x[j + 1].x : round_end;
        ranges2[i] = make_uint2(x.x, end);
        tile_cnt[kTileCntStride * i + 2] = x.y;
      }
    }
    carry += tot;
    __syncthreads();                   // s_x is refilled by the next round
  }
  const bool over = carry > (unsigned long long)capacity;
  if (over) {
    // same thread-to-entry mapping as the stores above, so these land after the ones they replace
    for (int base = 0; base < n_tiles; base += kScanRound) {
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) {
        const int i = base + 1024 * k + tid;
        if (i < n_tiles) ranges2[i] = make_uint2(0u, 0u);
      }
    }
  }
  if (tid == 0) {
    *K_out = (int64_t)carry;
    overflow[0] = over ? 1u : 0u;     // this binning
    if (over) overflow[2] = 1u;       // sticky until tsr_check reads it (spans graph replays)
  }
}

// Emission of (float32 z_F bits << 32 | face) into each overlapped tile's bucket.  One
// workgroup per visible-list segment, one lane per visible face of the segment (compacted,
// in pair order), each reading its 32-byte visible-list entry.  Small faces store at their
// recorded slot; larger faces take positions from the per-tile cursors, spread over the
// wave.  A position outside its tile's range (never expected) is not written and is reported
// through tsr_check.  Under tight binning a small face's skipped tiles carry kSkipSlot, and the
// larger faces repeat the projection's FP64 setup (the same code on the same inputs, so the same
// tile decisions) to list only the tiles the projection counted.
constexpr int kEmitU = 4;          // larger-face tiles per lane per expansion round of the emission

template <bool TIGHT>
__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ ranges,
                                              uint32_t* __restrict__ cursor, uint32_t* __restrict__ overflow,
                                              uint64_t* __restrict__ pairs, const uint32_t* __restrict__ vis_cnt,
                                              const uint32_t* __restrict__ vis_off, const VisEntry* __restrict__ vis_list,
                                              uint32_t* __restrict__ vis_dense, tsr_scene_dev sc,
                                              const float* __restrict__ poses, ViewTable vt, float z_near, float r_min) {
  const uint32_t nvis = vis_cnt[blockIdx.x];
  const bool mine = threadIdx.x < nvis;
  const uint4* ent = reinterpret_cast<const uint4*>(vis_list + (int64_t)blockIdx.x * kProjBlock + threadIdx.x);
  uint4 e0 = make_uint4(0u, 0u, 0u, 0u);
  if (mine) {
    e0 = ent[0];
    // the segment goes to its place in the dense list (done even when the pairs overflowed:
    // the backward uses it)
    vis_dense[vis_off[blockIdx.x] + threadIdx.x] = e0.x;
  }
  if (overflow[0]) return;
  const int tile0 = (int)e0.y;
  const int tw = (int)(e0.z & 1023u) + 1, th = (int)((e0.z >> 10) & 1023u) + 1, tiles_x = (int)(e0.z >> 20) + 1;
  const int ntiles = mine ? tw * th : 0;
  const uint64_t key = ((uint64_t)e0.w << 32) | (uint64_t)e0.x;
  if (ntiles > 0 && ntiles <= kSmallTiles) {
    // slots recorded during counting: plain stores
    const uint4 sl = ent[1];
    const uint32_t slv[4] = {sl.x, sl.y, sl.z, sl.w};
    bool bad = false;
#pragma unroll
    for (int i = 0; i < kSmallTiles; ++i)
      if (i < ntiles && slv[i] != kSkipSlot) {
        const int t = tile0 + (i / tw) * tiles_x + i % tw;
        const uint32_t pos = ranges[2 * t] + slv[i];
        if (pos < ranges[2 * t + 1]) pairs[pos] = key;
        else bad = true;
      }
    if (bad) atomicOr(&overflow[2], 2u);          // reported by tsr_check; nothing written
  }
  const int big = ntiles > kSmallTiles ? ntiles : 0;
  if (wave_max_int(big) == 0) return;
  const uint32_t key_hi = (uint32_t)(key >> 32), key_lo = (uint32_t)key;
  EdgeLines el{};
  int ltx0 = 0, lty0 = 0;      // view-local tile of tile0
  if constexpr (TIGHT) {
    if (big > 0) {
      const int64_t M = vt.n_faces;
      const int v = (int)((int64_t)e0.x / M);
      const int64_t m = (int64_t)e0.x - (int64_t)v * M;
      double R[9], t[3];
      load_pose(poses, v, R, t);
      int64_t vid[3];
      face_vertices(sc, m, vid);
      FaceSetup f;
      setup_face(sc, vid, R, t, vt.v[v], z_near, r_min, f);   // visible: it was listed by the projection
      face_normals(f);
      edge_lines(f, el);
      ltx0 = f.u0 >> 4;
      lty0 = f.v0 >> 4;
    }
  }
  // The larger faces' tiles spread over the wave (owner lane by binary search over the wave's
  // inclusive prefix of the counts), kEmitU items per lane per round: a round resolves its
  // items' tiles and keys, then issues all their cursor atomics (without a branch, so nothing
  // waits between them; under tight binning a tile the face does not cover adds 0 to its own
  // cursor), then stores, so that a face over hundreds of tiles waits on one atomic round trip
  // per kEmitU x 64 of its tiles rather than per 64 (1200x680 with 1M faces: the larger faces
  // took 12.7 us of the emission's 21: now 8.7).  Items past the last full round go one per
  // lane, with a branch around each atomic (repeating real items with adds of 0 to fill the
  // last round instead multiplied the atomics on the busiest cursors: 17 -> 22 us).
  const int lane = threadIdx.x & 63;
  int incl = big;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const int total = __shfl(incl, 63, 64);
  // item j of the wave: its tile, its key, and whether the face lists that tile
  auto item = [&](int j, int& t, uint64_t& key2) -> bool {
    int lo = 0, hi = 63;
#pragma unroll
    for (int st = 0; st < 6; ++st) {             // smallest lane with incl > j
      const int mid = (lo + hi) >> 1;
      if (__shfl(incl, mid, 64) > j) hi = mid; else lo = mid + 1;
    }
    const int owner = lo;
    const int i = j - (__shfl(incl, owner, 64) - __shfl(big, owner, 64));
    const int ot0 = __shfl(tile0, owner, 64), otw = __shfl(tw, owner, 64), otx = __shfl(tiles_x, owner, 64);
    const uint32_t khi = __shfl(key_hi, owner, 64), klo = __shfl(key_lo, owner, 64);
    bool keep = true;
    if constexpr (TIGHT) {
      EdgeLines oe;
      shfl_lines(el, owner, oe);
      const int ox = __shfl(ltx0, owner, 64), oy = __shfl(lty0, owner, 64);
      keep = tile_may_cover(oe, ox + i % otw, oy + i / otw);
    }
    t = ot0 + (i / otw) * otx + i % otw;
    key2 = ((uint64_t)khi << 32) | klo;
    return keep;
  };
  int base = 0;
  for (; base + kWave * kEmitU <= total; base += kWave * kEmitU) {
    int tt[kEmitU];
    uint64_t kk[kEmitU];
    bool ok[kEmitU];
#pragma unroll
    for (int u = 0; u < kEmitU; ++u) ok[u] = item(base + u * kWave + lane, tt[u], kk[u]);
    uint32_t r0[kEmitU], r1[kEmitU], slot[kEmitU];
#pragma unroll
    for (int u = 0; u < kEmitU; ++u) {
      r0[u] = ranges[2 * tt[u]];
      r1[u] = ranges[2 * tt[u] + 1];
      slot[u] = atomicAdd(&cursor[kTileCntStride * tt[u] + 2], ok[u] ? 1u : 0u);
    }
#pragma unroll
    for (int u = 0; u < kEmitU; ++u)
      if (ok[u]) {
        const uint32_t pos = r0[u] + slot[u];
        if (pos < r1[u]) pairs[pos] = kk[u];
        else atomicOr(&overflow[2], 2u);
      }
  }
  for (; base < total; base += kWave) {
    const int j = base + lane;
    int t;
    uint64_t key2;
    const bool keep = item(j, t, key2);
    if (j < total && keep) {
      const uint32_t pos = ranges[2 * t] + atomicAdd(&cursor[kTileCntStride * t + 2], 1u);
      if (pos < ranges[2 * t + 1]) pairs[pos] = key2;
      else atomicOr(&overflow[2], 2u);
    }
  }
}

// ---------------------------------------------------------------------------- per-tile sort
constexpr int kSortLds = 4096;     // keys sorted in one LDS pass (32 KiB)

__device__ __forceinline__ void bitonic_lds(uint64_t* s, int n2) {
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = s[i], b = s[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ int lower_bound_u64(const uint64_t* a, int n, uint64_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Value held by lane (lane ^ j), j in {1, 2, 4, 8, 16, 32}, without a trip through LDS: DPP
// inside 16-lane rows (quad permutes; half-row mirror i^7 followed by quad permute i^3 gives
// i^4; a row rotation by 8 is i^8), gfx950 permlane swaps across rows.  With the same
// register as both operands, v_permlane16_swap leaves rows (0,0,2,2) in its first result and
// (1,1,3,3) in its second; v_permlane32_swap leaves halves (0,0) and (1,1).  Every lane of
// the wave must be active; j must fold to a constant once the caller's loops are unrolled.
// Every source lane of these DPP patterns lies in its own row, so with bound_ctrl set no lane
// takes the "old" operand and the compiler needs no register for it.
__device__ __forceinline__ uint32_t lane_xor_u32(uint32_t x, int j) {
  const int lane = threadIdx.x & 63;
  const int xi = (int)x;
  switch (j) {
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0xB1, 0xF, 0xF, true);    // quad_perm [1,0,3,2]
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0x4E, 0xF, 0xF, true);    // quad_perm [2,3,0,1]
    case 4: {
      const int y = __builtin_amdgcn_update_dpp(0, xi, 0x141, 0xF, 0xF, true);           // row_half_mirror
      return (uint32_t)__builtin_amdgcn_update_dpp(0, y, 0x1B, 0xF, 0xF, true);          // quad_perm [3,2,1,0]
    }
    case 8: return (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0x128, 0xF, 0xF, true);   // row_ror:8
    case 16: {
      const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
      return (lane & 16) ? p[0] : p[1];
    }
    default: {
      const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
      return (lane & 32) ? p[0] : p[1];
    }
  }
}

__device__ __forceinline__ uint64_t lane_xor_u64(uint64_t x, int j) {
  const uint32_t lo = lane_xor_u32((uint32_t)x, j), hi = lane_xor_u32((uint32_t)(x >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}

// One compare-exchange of a bitonic network: key a at position e meets its partner b; the
// lower position of the pair keeps the minimum when the run of length kk ascends, the upper
// one when it descends.  b replaces a exactly when it is the key to keep: one 64-bit compare
// against a per-position flag (a function of lane bits and constants once unrolled) and a
// select, rather than forming both the minimum and the maximum.
__device__ __forceinline__ uint64_t bitonic_keep(uint64_t a, uint64_t b, int e, int j, int kk) {
  const bool keep_min = ((e & kk) == 0) == ((e & j) == 0);
  return ((b < a) == keep_min) ? b : a;
}

// Register bitonic sort of up to 64 * R keys held by one wave, lane-major (key e = lane * R + r):
// exchanges with j < R stay inside a lane's registers (a compare and two selects per key, no
// permute), the others pair lane with lane ^ (j / R) through lane_xor_u64.  For 512 keys that
// leaves 21 of the 45 stages crossing lanes, against 39 with the keys laid out r * 64 + lane.
template <int R>
__device__ __forceinline__ void wave_bitonic(uint64_t (&k)[R]) {
  const int lane = threadIdx.x & 63;
  constexpr int N = 64 * R;
#pragma unroll
  for (int kk = 2; kk <= N; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j < R) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (r & j) continue;
          const bool up = ((lane * R + r) & kk) == 0;
          const uint64_t a = k[r], b = k[r ^ j];
          if ((a > b) == up) {
            k[r] = b;
            k[r ^ j] = a;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) k[r] = bitonic_keep(k[r], lane_xor_u64(k[r], j / R), lane * R + r, j, kk);
      }
    }
  }
}

// Bitonic sort of 1024 keys by one workgroup of 256 threads, four keys per thread (key
// e = r * 256 + tid): partners within a wave via lane_xor_u64, partners in another wave of the
// same lane through LDS (double-buffered, one barrier per stage), partners in another
// register of the same thread locally.  `s` holds 2 x 1024 keys.  Ends with a barrier.
__device__ __forceinline__ void block_bitonic1024(uint64_t (&k)[4], uint64_t* s) {
  const int tid = threadIdx.x;
  int buf = 0;
#pragma unroll
  for (int kk = 2; kk <= 1024; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j >= 256) {
        const int rj = j >> 8;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (r & rj) continue;
          const bool up = ((r * 256 + tid) & kk) == 0;
          const uint64_t a = k[r], b = k[r ^ rj];
          if ((a > b) == up) {
            k[r] = b;
            k[r ^ rj] = a;
          }
        }
      } else if (j >= 64) {
        uint64_t* b = s + buf * 1024;
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r * 256 + tid] = k[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) k[r] = bitonic_keep(k[r], b[(r * 256 + tid) ^ j], r * 256 + tid, j, kk);
        buf ^= 1;
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) k[r] = bitonic_keep(k[r], lane_xor_u64(k[r], j), r * 256 + tid, j, kk);
      }
    }
  }
  __syncthreads();
}

template <int R>
__device__ __forceinline__ void wave_sort_tile(uint64_t* base, int n) {
  const int lane = threadIdx.x & 63;
  uint64_t k[R];
#pragma unroll
  for (int r = 0; r < R; ++r) k[r] = (lane * R + r < n) ? base[lane * R + r] : ~0ull;
  wave_bitonic<R>(k);
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (lane * R + r < n) base[lane * R + r] = k[r];
}

// Per-tile depth sort, ascending by (z bits, face), in one launch with two kinds of
// workgroups: the first kLongBlocks are persistent over the list of tiles longer than
// kWaveSortMax keys (built by k_scan_tiles), so they start first and overlap the rest; each
// remaining workgroup sorts four tiles, one wave each, in registers.
//   Long lists of up to kRegSortMax keys are sorted in registers by the whole workgroup
// (block_bitonic1024); up to kSortLds keys are bitonic-sorted in LDS; longer ones are sorted
// in LDS-sized chunks and merged pairwise in global memory through `temp` (keys are unique,
// so a rank by binary search places every key).
constexpr int kLongBlocks = 64;

__device__ __forceinline__ void sort_long_tiles(const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ long_cnt,
                                                const uint32_t* __restrict__ long_list, uint64_t* __restrict__ pairs,
                                                uint64_t* __restrict__ temp, uint64_t* s, uint32_t first) {
  const uint32_t nl = *long_cnt;
  for (uint32_t li = first; li < nl; li += kLongBlocks) {
  const int t = (int)long_list[li];
  const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
  const int n = (int)(end - start);
  uint64_t* base = pairs + start;
  if (n <= kRegSortMax) {
    static_assert(kRegSortMax == 1024, "block_bitonic1024 sorts 1024 keys");
    uint64_t k[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) k[r] = (r * 256 + (int)threadIdx.x < n) ? base[r * 256 + threadIdx.x] : ~0ull;
    block_bitonic1024(k, s);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (r * 256 + (int)threadIdx.x < n) base[r * 256 + threadIdx.x] = k[r];
    continue;
  }
  for (int c0 = 0; c0 < n; c0 += kSortLds) {
    const int cn = min(kSortLds, n - c0);
    int n2 = 1;
    while (n2 < cn) n2 <<= 1;
    for (int i = threadIdx.x; i < n2; i += blockDim.x) s[i] = i < cn ? base[c0 + i] : ~0ull;
    __syncthreads();
    bitonic_lds(s, n2);
    for (int i = threadIdx.x; i < cn; i += blockDim.x) base[c0 + i] = s[i];
    __syncthreads();
  }
  if (n <= kSortLds) continue;
  uint64_t* src = base;
  uint64_t* dst = temp + start;
  for (int width = kSortLds; width < n; width <<= 1) {
    __threadfence();
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int run = i / width;
      const int pair_lo = (run & ~1) * width;
      const int a_lo = pair_lo, a_n = min(width, n - a_lo);
      const int b_lo = pair_lo + width, b_n = max(0, min(width, n - b_lo));
      const uint64_t x = src[i];
      int outpos;
      if ((run & 1) == 0) outpos = pair_lo + (i - a_lo) + lower_bound_u64(src + b_lo, b_n, x);
      else outpos = pair_lo + (i - b_lo) + lower_bound_u64(src + a_lo, a_n, x);
      dst[outpos] = x;
    }
    uint64_t* tmp = src;
    src = dst;
    dst = tmp;
  }
  __threadfence();
  __syncthreads();
  if (src != base)
    for (int i = threadIdx.x; i < n; i += blockDim.x) base[i] = src[i];
  __syncthreads();
  }
}

// Workgroup 0 builds the longest-first tile order when `order` is given (running beside the
// sorts); the next kLongBlocks sort the long lists; the rest sort one short tile list per wave.
__global__ __launch_bounds__(256) void k_tile_sort(const uint32_t* __restrict__ ranges, int n_tiles,
                                                   uint64_t* __restrict__ pairs, const uint32_t* __restrict__ long_cnt,
                                                   const uint32_t* __restrict__ long_list, uint64_t* __restrict__ temp,
                                                   int* __restrict__ order) {
  __shared__ uint64_t s[kSortLds];
  static_assert(kOrderBuckets * sizeof(uint32_t) + 16 * sizeof(uint64_t) <= sizeof(s), "order scratch in LDS");
  if (blockIdx.x == 0) {
    if (order)
      build_tile_order(ranges, n_tiles, order, reinterpret_cast<uint32_t*>(s),
                       reinterpret_cast<unsigned long long*>(s + kOrderBuckets / 2));
    return;
  }
  if (blockIdx.x <= kLongBlocks) {
    sort_long_tiles(ranges, long_cnt, long_list, pairs, temp, s, blockIdx.x - 1);
    return;
  }
  const int t = (int)(blockIdx.x - 1 - kLongBlocks) * 4 + (int)(threadIdx.x >> 6);
  if (t >= n_tiles) return;
  const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
  const int n = (int)(end - start);
  if (n <= 1 || n > kWaveSortMax) return;
  static_assert(kWaveSortMax == 512, "the one-wave sort holds at most 8 keys per lane");
  uint64_t* base = pairs + start;
  if (n <= 64) wave_sort_tile<1>(base, n);
  else if (n <= 128) wave_sort_tile<2>(base, n);
  else if (n <= 256) wave_sort_tile<4>(base, n);
  else wave_sort_tile<8>(base, n);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------- launchers

static inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_ws_init(char* ws, hipStream_t st) {
  TSR_LAUNCH("ws_init", k_fill_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(ws), (int64_t)64, 0u);
  return hipGetLastError();
}

// Projected image-space area (pixels^2, half the absolute cross product of the projected
// edges) of every (view, face) that survives the near-plane and inradius culls and overlaps the
// image, 0 for the others; the same FP64 setup as the projection.  Thread idx = v * M + m.
__global__ __launch_bounds__(256) void k_face_area(tsr_scene_dev sc, const float* __restrict__ poses, ViewTable vt,
                                                   float z_near, float r_min, float* __restrict__ area) {
  const int64_t M = vt.n_faces;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)vt.n_views * M) return;
  const int v = (int)(idx / M);
  const int64_t m = idx - (int64_t)v * M;
  double R[9], t[3];
  load_pose(poses, v, R, t);
  int64_t vid[3];
  face_vertices(sc, m, vid);
  FaceSetup f;
  const bool ok = setup_face(sc, vid, R, t, vt.v[v], z_near, r_min, f);
  area[idx] = ok ? (float)(0.5 * f.area2) : 0.f;
}

hipError_t launch_face_area(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                            float* area, hipStream_t st) {
  const int64_t n = (int64_t)vt.n_views * vt.n_faces;
  if (n > 0)
    TSR_LAUNCH("face_area", k_face_area, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sc, poses, vt,
               p.z_near, p.r_min, area);
  return hipGetLastError();
}

hipError_t launch_bin(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                      const WsLayout& L, char* ws, bool sort, hipStream_t st) {
  uint32_t* counts = reinterpret_cast<uint32_t*>(ws + L.counts);
  float* records = reinterpret_cast<float*>(ws + L.records);
  uint32_t* tile_cnt = reinterpret_cast<uint32_t*>(ws + L.tile_cnt);
  uint32_t* ranges = reinterpret_cast<uint32_t*>(ws + L.ranges);
  int64_t* K = reinterpret_cast<int64_t*>(ws + L.hdr_k);
  uint32_t* overflow = reinterpret_cast<uint32_t*>(ws + L.hdr_overflow);
  uint64_t* pairs = reinterpret_cast<uint64_t*>(ws + L.pairs);
  uint64_t* temp = reinterpret_cast<uint64_t*>(ws + L.temp);
  const int64_t nf = (int64_t)vt.n_views * vt.n_faces;

  uint32_t* vis_cnt = reinterpret_cast<uint32_t*>(ws + L.vis_cnt);
  VisEntry* vis_list = reinterpret_cast<VisEntry*>(ws + L.vis_list);
  uint32_t* long_cnt = reinterpret_cast<uint32_t*>(ws + L.long_cnt);
  uint32_t* long_list = reinterpret_cast<uint32_t*>(ws + L.long_list);
  // the tile counters and the long-tile counter are contiguous: one fill
  const int64_t n_cnt = kTileCntStride * (int64_t)vt.n_tiles + 1;
  TSR_LAUNCH("fill_tiles", k_fill_u32, dim3(grid_for(n_cnt, 256)), dim3(256), 0, st, tile_cnt, n_cnt, 0u);
  if (nf > 0) {
    // one pre-test round per projection workgroup for a single view, four for several
#define TSR_PROJECT(T, R)                                                                                   \
  TSR_LAUNCH("project", (k_project<T, R>), dim3(grid_for(nf, (int64_t)R * kProjBlock)), dim3(kProjBlock), 0, st, sc, \
             poses, vt, p.z_near, p.r_min, p.sigma, p.perspective, counts, records, tile_cnt, vis_cnt, vis_list)
    if (proj_rounds(vt.n_views) == 1) {
      if (p.tight_tiles) TSR_PROJECT(true, 1);
      else TSR_PROJECT(false, 1);
    } else {
      if (p.tight_tiles) TSR_PROJECT(true, 4);
      else TSR_PROJECT(false, 4);
    }
#undef TSR_PROJECT
  }
  uint32_t* vis_off = reinterpret_cast<uint32_t*>(ws + L.vis_off);
  uint32_t* vis_total = reinterpret_cast<uint32_t*>(ws + L.vis_total);
  uint32_t* vis_dense = reinterpret_cast<uint32_t*>(ws + L.vis_dense);
  const int n_seg = (int)proj_segments(nf, vt.n_views);
  TSR_LAUNCH("scan_tiles", k_scan_tiles, dim3(2), dim3(1024), 0, st, tile_cnt, ranges, vt.n_tiles,
                     sort ? L.capacity : (int64_t)0x7fffffffffffffffll, K, overflow, vis_cnt, vis_off, vis_total,
                     n_seg, long_cnt, long_list);
  if (!sort) return hipGetLastError();
  if (nf > 0) {
    if (p.tight_tiles)
      TSR_LAUNCH("emit", k_emit<true>, dim3(n_seg), dim3(kProjBlock), 0, st, ranges, tile_cnt,
                 overflow, pairs, vis_cnt, vis_off, vis_list, vis_dense, sc, poses, vt, p.z_near, p.r_min);
    else
      TSR_LAUNCH("emit", k_emit<false>, dim3(n_seg), dim3(kProjBlock), 0, st, ranges, tile_cnt,
                 overflow, pairs, vis_cnt, vis_off, vis_list, vis_dense, sc, poses, vt, p.z_near, p.r_min);
  }
  // small tile counts: the order is built beside the sorts (hidden behind them); larger ones by
  // the backward set-up, and only for schedules that use it
  int* order = vt.n_tiles <= kOrderInSortMax ? reinterpret_cast<int*>(ws + L.order) : nullptr;
  TSR_LAUNCH("tile_sort", k_tile_sort, dim3(1 + kLongBlocks + grid_for(vt.n_tiles, 4)), dim3(256), 0, st, ranges,
             vt.n_tiles, pairs, long_cnt, long_list, temp, order);
  return hipGetLastError();
}

}  // namespace tsr
