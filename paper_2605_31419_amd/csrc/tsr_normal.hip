// Normal supervision of mapping (Sec. 3.4): sensor normals from depth and the normal loss
// E_norm = mean over valid pixels of (1 - N(p) . N_bar(p)), with N the rendered normal map.
//
// The rendered map composites each face's world unit normal like a colour that is constant
// over the face, then rotates it into the camera frame: N = R_CW N_w.  Two forms:
//
// The normal step on its own (launch_train_normal) runs the rasterizer on the soup with every
// vertex colour set to its face normal (binning, forward, backward), and adds around it:
//   k_normal_colours  face normals (FP64) written as vertex colours;
//   k_count_valid     valid target pixels per view (a target normal of 0 marks an invalid one);
//   k_normal_seeds    N = R N_w, the loss sums, the colour seed dE/dN_w = R^T dE/dN and the
//                     rotation term sum_p N x dE/dN of the pose gradient;
//   k_normal_chain    the face-normal gradient (sum of its vertices' colour gradients) through
//                     the normalised cross product into the vertex positions;
//   k_normal_finish   per-view loss and the rotation term added to the pose gradient.
//
// The mapping step (launch_train_mapping) carries the normals as three more channels of the
// photometric walks on the scene's own binning: k_face_normals writes them per face, the
// forward compares N with the target per pixel and leaves per-wave sums that k_normal_reduce
// turns into each view's valid count, loss and rotation term, the backward forms the seeds from
// the target itself and sums dE/dn_F per face, and k_normal_chain_faces takes that through the
// normalised cross product into the position gradients.
#include "tsr_device.h"
#include "tsr_internal.h"

namespace tsr {

constexpr int kNormBlocksPerView = 256;

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ void load_face(const float* __restrict__ pos, int64_t N, int64_t m, double e1[3],
                                          double e2[3]) {
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double p0 = pos[ax * N + 3 * m], p1 = pos[ax * N + 3 * m + 1], p2 = pos[ax * N + 3 * m + 2];
    e1[ax] = p1 - p0;
    e2[ax] = p2 - p0;
  }
}

__global__ __launch_bounds__(256) void k_normal_colours(const float* __restrict__ pos, int64_t N, int64_t M,
                                                        float* __restrict__ col) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double e1[3], e2[3], c[3];
  load_face(pos, N, m, e1, e2);
  cross3(e1, e2, c);
  const double L = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  const double il = L > 0.0 ? 1.0 / L : 0.0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const float n = (float)(c[ax] * il);
    col[ax * N + 3 * m] = n;
    col[ax * N + 3 * m + 1] = n;
    col[ax * N + 3 * m + 2] = n;
  }
}

// Sensor normals: central differences of the back-projected points, FP64.
__global__ __launch_bounds__(256) void k_sensor_normals(const float* __restrict__ depth, ViewTable vt,
                                                        float* __restrict__ normals) {
  const int v = blockIdx.y;
  const ViewDesc vd = vt.v[v];
  const int64_t P = (int64_t)vd.width * vd.height;
  const float* d = depth + vd.pix_off;
  float* out = normals + 3 * vd.pix_off;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(i % vd.width), y = (int)(i / vd.width);
    double n[3] = {0.0, 0.0, 0.0};
    if (u >= 1 && u <= vd.width - 2 && y >= 1 && y <= vd.height - 2) {
      const double dc = d[i], dl = d[i - 1], dr = d[i + 1], du = d[i - vd.width], dd = d[i + vd.width];
      if (dc > 0.0 && dl > 0.0 && dr > 0.0 && du > 0.0 && dd > 0.0) {
        const double ifx = 1.0 / (double)vd.fx, ify = 1.0 / (double)vd.fy;
        auto pt = [&](double z, int uu, int vv, double p[3]) {
          p[0] = z * ((double)uu - (double)vd.cx) * ifx;
          p[1] = z * ((double)vv - (double)vd.cy) * ify;
          p[2] = z;
        };
        double pl[3], pr[3], pu[3], pd[3], gx[3], gy[3], c[3];
        pt(dl, u - 1, y, pl);
        pt(dr, u + 1, y, pr);
        pt(du, u, y - 1, pu);
        pt(dd, u, y + 1, pd);
        for (int a = 0; a < 3; ++a) {
          gx[a] = 0.5 * (pr[a] - pl[a]);
          gy[a] = 0.5 * (pd[a] - pu[a]);
        }
        cross3(gx, gy, c);
        const double L = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (L > 0.0)
          for (int a = 0; a < 3; ++a) n[a] = c[a] / L;
      }
    }
    for (int a = 0; a < 3; ++a) out[a * P + i] = (float)n[a];
  }
}

__device__ __forceinline__ bool valid_target(const float* t, int64_t P, int64_t i) {
  return t[i] != 0.f || t[P + i] != 0.f || t[2 * P + i] != 0.f;
}

template <class T>
__device__ __forceinline__ T block_sum256(T x, T* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_count_valid(ViewTable vt, const float* __restrict__ target,
                                                     uint32_t* __restrict__ count) {
  __shared__ uint32_t red[4];
  const int v = blockIdx.y;
  const ViewDesc vd = vt.v[v];
  const int64_t P = (int64_t)vd.width * vd.height;
  const float* t = target + 3 * vd.pix_off;
  uint32_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x)
    c += valid_target(t, P, i) ? 1u : 0u;
  c = block_sum256(c, red);
  if (threadIdx.x == 0 && c) atomicAdd(&count[v], c);
}

__global__ __launch_bounds__(256) void k_normal_seeds(ViewTable vt, const float* __restrict__ poses,
                                                      const float* __restrict__ nw, const float* __restrict__ target,
                                                      const uint32_t* __restrict__ count, float w_norm,
                                                      float* __restrict__ normal_map, float* __restrict__ seed,
                                                      double* __restrict__ acc) {
  __shared__ double red[4];
  const int v = blockIdx.y;
  const ViewDesc vd = vt.v[v];
  const int64_t P = (int64_t)vd.width * vd.height;
  float R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = poses[12 * v + k];
  const float inv = count[v] ? w_norm / (float)count[v] : 0.f;
  const float* src = nw + 3 * vd.pix_off;
  const float* t = target + 3 * vd.pix_off;
  float* nm = normal_map ? normal_map + 3 * vd.pix_off : nullptr;
  float* sd = seed + 3 * vd.pix_off;
  double l = 0.0, r0 = 0.0, r1 = 0.0, r2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    const float a0 = src[i], a1 = src[P + i], a2 = src[2 * P + i];
    const float n0 = R[0] * a0 + R[1] * a1 + R[2] * a2;
    const float n1 = R[3] * a0 + R[4] * a1 + R[5] * a2;
    const float n2 = R[6] * a0 + R[7] * a1 + R[8] * a2;
    if (nm) {
      nm[i] = n0;
      nm[P + i] = n1;
      nm[2 * P + i] = n2;
    }
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
    if (valid_target(t, P, i)) {
      const float b0 = t[i], b1 = t[P + i], b2 = t[2 * P + i];
      l += (double)(1.f - (n0 * b0 + n1 * b1 + n2 * b2));
      g0 = -inv * b0;
      g1 = -inv * b1;
      g2 = -inv * b2;
      r0 += (double)(n1 * g2 - n2 * g1);
      r1 += (double)(n2 * g0 - n0 * g2);
      r2 += (double)(n0 * g1 - n1 * g0);
    }
    // dE/dN_w = R^T dE/dN
    sd[i] = R[0] * g0 + R[3] * g1 + R[6] * g2;
    sd[P + i] = R[1] * g0 + R[4] * g1 + R[7] * g2;
    sd[2 * P + i] = R[2] * g0 + R[5] * g1 + R[8] * g2;
  }
  l = block_sum256(l, red);
  r0 = block_sum256(r0, red);
  r1 = block_sum256(r1, red);
  r2 = block_sum256(r2, red);
  if (threadIdx.x == 0) {
    atomicAdd(&acc[4 * v], l);
    atomicAdd(&acc[4 * v + 1], r0);
    atomicAdd(&acc[4 * v + 2], r1);
    atomicAdd(&acc[4 * v + 3], r2);
  }
}

// dE/dn_F (the sum of the face's three vertex-colour gradients) through n = c / |c|,
// c = e1 x e2: dE/dc = (I - n n^T) dE/dn / |c|, dE/de1 = e2 x dE/dc, dE/de2 = dE/dc x e1.
__global__ __launch_bounds__(256) void k_normal_chain(const float* __restrict__ pos, int64_t N, int64_t M,
                                                      const float* __restrict__ gcol, float* __restrict__ grad_pos) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double e1[3], e2[3], c[3], gn[3];
  load_face(pos, N, m, e1, e2);
  cross3(e1, e2, c);
  const double L = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  if (!(L > 0.0)) return;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
    gn[ax] = (double)gcol[ax * N + 3 * m] + (double)gcol[ax * N + 3 * m + 1] + (double)gcol[ax * N + 3 * m + 2];
  double n[3], gc[3], g1[3], g2[3];
  for (int ax = 0; ax < 3; ++ax) n[ax] = c[ax] / L;
  const double dn = n[0] * gn[0] + n[1] * gn[1] + n[2] * gn[2];
  for (int ax = 0; ax < 3; ++ax) gc[ax] = (gn[ax] - n[ax] * dn) / L;
  cross3(e2, gc, g1);
  cross3(gc, e1, g2);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    float* g = grad_pos + ax * N + 3 * m;
    g[0] = (float)((double)g[0] - g1[ax] - g2[ax]);
    g[1] = (float)((double)g[1] + g1[ax]);
    g[2] = (float)((double)g[2] + g2[ax]);
  }
}

__global__ void k_normal_finish(int n_views, const uint32_t* __restrict__ count, const double* __restrict__ acc,
                                float w_norm, float* __restrict__ loss, float* __restrict__ grad_pose) {
  const int v = threadIdx.x;
  if (v >= n_views) return;
  if (loss) loss[v] = count[v] ? (float)((double)w_norm * acc[4 * v] / (double)count[v]) : 0.f;
  if (grad_pose)
    for (int k = 0; k < 3; ++k) grad_pose[6 * v + 3 + k] += (float)acc[4 * v + 1 + k];
}

// Face normals of the normal channels: [M] float4 (x, y, z, 0), FP64 arithmetic; a degenerate
// face gets 0.  Also zeroes the face's normal-gradient accumulator.
__global__ __launch_bounds__(256) void k_face_normals(const float* __restrict__ pos, int64_t N, int64_t M,
                                                      float4* __restrict__ nrm, float4* __restrict__ gacc) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  gacc[m] = make_float4(0.f, 0.f, 0.f, 0.f);
  double e1[3], e2[3], c[3];
  load_face(pos, N, m, e1, e2);
  cross3(e1, e2, c);
  const double L = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  const double il = L > 0.0 ? 1.0 / L : 0.0;
  nrm[m] = make_float4((float)(c[0] * il), (float)(c[1] * il), (float)(c[2] * il), 0.f);
}

// dE/dn_F of the normal channels (summed over the views by the backward walk) through the
// normalised cross product, added to the soup's vertex gradients (as k_normal_chain).
__global__ __launch_bounds__(256) void k_normal_chain_faces(const float* __restrict__ pos, int64_t N, int64_t M,
                                                            const float4* __restrict__ gacc,
                                                            float* __restrict__ grad_pos) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double e1[3], e2[3], c[3];
  load_face(pos, N, m, e1, e2);
  cross3(e1, e2, c);
  const double L = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  if (!(L > 0.0)) return;
  const float4 g = gacc[m];
  const double gn[3] = {(double)g.x, (double)g.y, (double)g.z};
  double n[3], gc[3], g1[3], g2[3];
  for (int ax = 0; ax < 3; ++ax) n[ax] = c[ax] / L;
  const double dn = n[0] * gn[0] + n[1] * gn[1] + n[2] * gn[2];
  for (int ax = 0; ax < 3; ++ax) gc[ax] = (gn[ax] - n[ax] * dn) / L;
  cross3(e2, gc, g1);
  cross3(gc, e1, g2);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    float* gp = grad_pos + ax * N + 3 * m;
    gp[0] = (float)((double)gp[0] - g1[ax] - g2[ax]);
    gp[1] = (float)((double)gp[1] + g1[ax]);
    gp[2] = (float)((double)gp[2] + g2[ax]);
  }
}

__global__ void k_zero_words(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t launch_sensor_normals(const ViewTable& vt, const float* depth, float* normals, hipStream_t st) {
  TSR_LAUNCH("sensor_normals", k_sensor_normals, dim3(kNormBlocksPerView, vt.n_views), dim3(256), 0, st, depth, vt,
             normals);
  return hipGetLastError();
}

NormalScratch normal_scratch(int64_t n_vertices, int64_t n_pixels) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  NormalScratch z;
  z.col = 0;
  z.gcol = up(z.col + sizeof(float) * 3 * (size_t)n_vertices);
  z.nw = up(z.gcol + sizeof(float) * 3 * (size_t)n_vertices);
  z.seed = up(z.nw + sizeof(float) * 3 * (size_t)n_pixels);
  z.depth = up(z.seed + sizeof(float) * 3 * (size_t)n_pixels);
  z.zeros = up(z.depth + sizeof(float) * (size_t)n_pixels);
  z.gpos = up(z.zeros + sizeof(float) * (size_t)n_pixels);
  z.gopa = up(z.gpos + sizeof(float) * 3 * (size_t)n_vertices);
  z.gpose = up(z.gopa + sizeof(float) * (size_t)n_vertices);
  z.count = up(z.gpose + sizeof(float) * 6 * TSR_MAX_VIEWS);
  z.acc = up(z.count + sizeof(uint32_t) * TSR_MAX_VIEWS);
  z.total = up(z.acc + sizeof(double) * 4 * TSR_MAX_VIEWS);
  return z;
}

__global__ void k_add_f32(float* __restrict__ dst, const float* __restrict__ src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

hipError_t launch_train_normal(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                               const WsLayout& L, char* ws, const float* target, float w_norm, float* normal_map,
                               float* loss, float* grad_pos, float* grad_opa, float* grad_pose, bool accumulate,
                               char* scratch, int64_t n_pixels, hipStream_t st) {
  const NormalScratch z = normal_scratch(sc.n_vertices, n_pixels);
  // accumulating: the gradients go to scratch first and are added to the caller's at the end
  float* const out_pos = grad_pos;
  float* const out_opa = grad_opa;
  float* const out_pose = grad_pose;
  if (accumulate) {
    if (grad_pos) grad_pos = reinterpret_cast<float*>(scratch + z.gpos);
    if (grad_opa) grad_opa = reinterpret_cast<float*>(scratch + z.gopa);
    if (grad_pose) grad_pose = reinterpret_cast<float*>(scratch + z.gpose);
  }
  float* col = reinterpret_cast<float*>(scratch + z.col);
  float* gcol = reinterpret_cast<float*>(scratch + z.gcol);
  float* nw = reinterpret_cast<float*>(scratch + z.nw);
  float* seed = reinterpret_cast<float*>(scratch + z.seed);
  float* dep = reinterpret_cast<float*>(scratch + z.depth);
  float* zeros = reinterpret_cast<float*>(scratch + z.zeros);
  uint32_t* count = reinterpret_cast<uint32_t*>(scratch + z.count);
  double* acc = reinterpret_cast<double*>(scratch + z.acc);
  const int64_t M = sc.n_faces, N = sc.n_vertices;
  const unsigned fb = (unsigned)((M + 255) / 256);
  if (accumulate && N > 3 * M) {
    // the backward writes the vertices of the faces only: clear the rest of the staged
    // gradients so that adding them leaves the caller's extra vertices unchanged
    if (grad_pos)
      TSR_LAUNCH("zero_words", k_zero_words, dim3(1024), dim3(256), 0, st, reinterpret_cast<uint32_t*>(grad_pos), 3 * N);
    if (grad_opa)
      TSR_LAUNCH("zero_words", k_zero_words, dim3(1024), dim3(256), 0, st, reinterpret_cast<uint32_t*>(grad_opa), N);
  }
  // clear the gradient-free depth seed, the valid counts and the FP64 sums
  TSR_LAUNCH("zero_words", k_zero_words, dim3(1024), dim3(256), 0, st, reinterpret_cast<uint32_t*>(zeros), n_pixels);
  TSR_LAUNCH("zero_words", k_zero_words, dim3(1), dim3(256), 0, st, count,
             (int64_t)((z.total - z.count) / sizeof(uint32_t)));
  if (M > 0) TSR_LAUNCH("normal_colours", k_normal_colours, dim3(fb), dim3(256), 0, st, sc.pos, N, M, col);
  tsr_scene_dev sn = sc;
  sn.col = col;
  sn.grad_face_sigma = nullptr;     // this loss renders with the exponents but does not return their gradient
  hipError_t e = launch_bin(sn, poses, vt, p, L, ws, true, st);
  if (e != hipSuccess) return e;
  e = launch_forward(vt, p, L, ws, nw, dep, nullptr, st);
  if (e != hipSuccess) return e;
  const dim3 pg(kNormBlocksPerView, vt.n_views);
  TSR_LAUNCH("count_valid", k_count_valid, pg, dim3(256), 0, st, vt, target, count);
  TSR_LAUNCH("normal_seeds", k_normal_seeds, pg, dim3(256), 0, st, vt, poses, nw, target, count, w_norm, normal_map,
             seed, acc);
  TrainSchedule sched{0, 0, 0};
  e = launch_backward(sn, poses, vt, p, L, ws, seed, zeros, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                      nullptr, grad_pos, grad_pos ? gcol : nullptr, grad_opa, grad_pose, false, sched, st, nullptr, true);
  if (e != hipSuccess) return e;
  if (grad_pos && M > 0)
    TSR_LAUNCH("normal_chain", k_normal_chain, dim3(fb), dim3(256), 0, st, sc.pos, N, M, gcol, grad_pos);
  TSR_LAUNCH("normal_finish", k_normal_finish, dim3(1), dim3(64), 0, st, vt.n_views, count, acc, w_norm, loss,
             grad_pose);
  if (accumulate) {
    const unsigned vb = (unsigned)std::min<int64_t>((3 * N + 255) / 256, 4096);
    if (out_pos && N > 0) TSR_LAUNCH("add_grads", k_add_f32, dim3(vb), dim3(256), 0, st, out_pos, grad_pos, 3 * N);
    if (out_opa && N > 0) TSR_LAUNCH("add_grads", k_add_f32, dim3(vb), dim3(256), 0, st, out_opa, grad_opa, N);
    if (out_pose)
      TSR_LAUNCH("add_grads", k_add_f32, dim3(1), dim3(256), 0, st, out_pose, grad_pose, (int64_t)6 * vt.n_views);
  }
  return hipGetLastError();
}

MappingScratch mapping_scratch(size_t ssim_bytes, int64_t n_faces, int64_t n_tiles) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  MappingScratch z;
  z.nrm = up(ssim_bytes);
  z.gacc = up(z.nrm + 16 * (size_t)n_faces);
  z.part = up(z.gacc + 16 * (size_t)n_faces);
  z.count = up(z.part + sizeof(float) * kNormalPart * kTileQuads * (size_t)n_tiles);
  z.acc = up(z.count + sizeof(uint32_t) * TSR_MAX_VIEWS);
  z.total = up(z.acc + sizeof(double) * 4 * TSR_MAX_VIEWS);
  return z;
}

// Per view, the forward's per-wave normal-loss sums in FP64: the valid-pixel count, the loss
// sum, and the rotation term sum_p N x dE/dN = -(w_norm / count) sum_p N x N_bar, in the layout
// k_normal_finish reads.  One 256-thread workgroup per view, four slots per thread in flight;
// overwrites count and acc.
__global__ __launch_bounds__(256) void k_normal_reduce(ViewTable vt, const float* __restrict__ part, float w_norm,
                                                       uint32_t* __restrict__ count, double* __restrict__ acc) {
  __shared__ double red[4];
  const int v = blockIdx.x;
  const ViewDesc vd = vt.v[v];
  const int64_t w0 = (int64_t)vd.tile_off * kTileQuads;
  const int64_t w1 = w0 + (int64_t)vd.tiles_x * vd.tiles_y * kTileQuads;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  static_assert(kNormalPart == 8, "a slot is two float4");
  for (int64_t base = w0; base < w1; base += 4 * 256) {
    float4 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t w = base + u * 256 + threadIdx.x;
      const float4* p = reinterpret_cast<const float4*>(part + kNormalPart * w);
      a[u] = w < w1 ? p[0] : make_float4(0.f, 0.f, 0.f, 0.f);
      b[u] = w < w1 ? p[1] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s[0] += (double)a[u].x;
      s[1] += (double)a[u].y;
      s[2] += (double)a[u].z;
      s[3] += (double)a[u].w;
      s[4] += (double)b[u].x;
    }
  }
  double tot[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) tot[k] = block_sum256(s[k], red);
  if (threadIdx.x == 0) {
    const uint32_t cn = (uint32_t)tot[0];
    const float inv = cn ? w_norm / (float)cn : 0.f;
    count[v] = cn;
    acc[4 * v] = tot[1];
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[4 * v + 1 + k] = -(double)inv * tot[2 + k];
  }
}

// The whole mapping energy on the binning in `ws` (made with the scene's colours): one
// forward that also composites the world normal map, the photometric / depth seeds and the
// normal seeds, one backward that takes both, then the normal-to-vertex chain and the normal
// loss's rotation term of the pose gradient.
hipError_t launch_train_mapping(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                                const WsLayout& L, char* ws, const SsimTable& t, const float* target_color,
                                const float* target_depth, const float* target_normals, float w_ssim, float w_norm,
                                float* color, float* depth, float* trans, float* normal_map, float* loss,
                                float* loss_norm, float* grad_pos, float* grad_col, float* grad_opa,
                                float* grad_pose, char* scratch, hipStream_t st) {
  const MappingScratch z = mapping_scratch(ssim_scratch_bytes(t), sc.n_faces, vt.n_tiles);
  float4* nrm = reinterpret_cast<float4*>(scratch + z.nrm);
  float4* gacc = reinterpret_cast<float4*>(scratch + z.gacc);
  float* part = reinterpret_cast<float*>(scratch + z.part);
  uint32_t* count = reinterpret_cast<uint32_t*>(scratch + z.count);
  double* acc = reinterpret_cast<double*>(scratch + z.acc);
  const int64_t M = sc.n_faces, N = sc.n_vertices;
  const unsigned fb = (unsigned)std::max<int64_t>((M + 255) / 256, 1);
  // face normals, and the per-face normal gradients set to zero (every other scratch entry is
  // written before it is read)
  if (M > 0) TSR_LAUNCH("face_normals", k_face_normals, dim3(fb), dim3(256), 0, st, sc.pos, N, M, nrm, gacc);
  const NormalChannels fc{reinterpret_cast<const float*>(nrm), normal_map, nullptr, poses, target_normals, nullptr,
                          part, w_norm};
  hipError_t e = launch_forward(vt, p, L, ws, color, depth, trans, st, &fc);
  if (e != hipSuccess) return e;
  TSR_LAUNCH("normal_reduce", k_normal_reduce, dim3(vt.n_views), dim3(256), 0, st, vt, part, w_norm, count, acc);
  float *gc = nullptr, *gd = nullptr;
  e = launch_photo_seeds(t, color, target_color, depth, target_depth, w_ssim, p.w_color, p.w_depth, loss, scratch,
                         &gc, &gd, st);
  if (e != hipSuccess) return e;
  const NormalChannels bc{reinterpret_cast<const float*>(nrm), nullptr, reinterpret_cast<float*>(gacc), poses,
                          target_normals, count, nullptr, w_norm};
  TrainSchedule sched{0, 0, 0};
  e = launch_backward(sc, poses, vt, p, L, ws, gc, gd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                      grad_pos, grad_col, grad_opa, grad_pose, false, sched, st, &bc, true);
  if (e != hipSuccess) return e;
  if (grad_pos && M > 0)
    TSR_LAUNCH("normal_chain", k_normal_chain_faces, dim3(fb), dim3(256), 0, st, sc.pos, N, M, gacc, grad_pos);
  TSR_LAUNCH("normal_finish", k_normal_finish, dim3(1), dim3(64), 0, st, vt.n_views, count, acc, w_norm, loss_norm,
             grad_pose);
  return hipGetLastError();
}

}  // namespace tsr
