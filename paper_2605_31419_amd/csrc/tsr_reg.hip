// Equilateral regulariser E_equi (Sec. 3.4, eq. 14): the mean over faces of the mean over the
// three corners of (cos theta - 1/2)^2, cos theta the dot product of the unit edge vectors
// leaving the corner, and its gradient with respect to the vertex positions.  A face with a
// zero-length edge contributes 0 and gets no gradient (its angles are undefined).
//
// One thread per face; the per-face arithmetic runs in FP64 with three square roots and three
// divisions (FP64 division is a long instruction sequence, so the unit edges and the gradient
// terms multiply by the reciprocal lengths), and the loss is summed per workgroup in FP64.
#include <mutex>

#include "tsr_device.h"
#include "tsr_internal.h"

namespace tsr {

constexpr int kEquiBlock = 256;

__global__ __launch_bounds__(kEquiBlock) void k_equi(const float* __restrict__ pos, int64_t N,
                                                     const int32_t* __restrict__ faces, int64_t M, double gscale,
                                                     int accumulate, float* __restrict__ grad,
                                                     double* __restrict__ partial) {
  __shared__ double red[kEquiBlock / 64];
  const int64_t m = (int64_t)blockIdx.x * kEquiBlock + threadIdx.x;
  double loss = 0.0;
  if (m < M) {
    int64_t vid[3];
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      vid[k] = faces ? (int64_t)faces[3 * m + k] : 3 * m + k;
      ok = ok && vid[k] >= 0 && vid[k] < N;
    }
    double p[3][3];
    if (ok) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) p[k][ax] = (double)pos[ax * N + vid[k]];
    }
    // edges e_k = p[k+1] - p[k] and their lengths
    double e[3][3], len[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) e[k][ax] = ok ? p[(k + 1) % 3][ax] - p[k][ax] : 0.0;
      len[k] = sqrt(e[k][0] * e[k][0] + e[k][1] * e[k][1] + e[k][2] * e[k][2]);
    }
    ok = ok && len[0] > 0.0 && len[1] > 0.0 && len[2] > 0.0;
    double g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (ok) {
      double il[3], h[3][3];     // reciprocal edge lengths (three divisions per face), unit edges
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        il[k] = 1.0 / len[k];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) h[k][ax] = e[k][ax] * il[k];
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // corner k: towards b = k+1 along +h[k] (length len[k]), towards c = k+2 along
        // -h[k+2] (length len[k+2])
        const int kb = (k + 1) % 3, kc = (k + 2) % 3;
        double uh[3], vh[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          uh[ax] = h[k][ax];
          vh[ax] = -h[kc][ax];
        }
        const double c = uh[0] * vh[0] + uh[1] * vh[1] + uh[2] * vh[2];
        loss += (c - 0.5) * (c - 0.5);
        const double s = gscale * (c - 0.5);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const double db = s * (vh[ax] - c * uh[ax]) * il[k];
          const double dc = s * (uh[ax] - c * vh[ax]) * il[kc];
          g[kb][ax] += db;
          g[kc][ax] += dc;
          g[k][ax] -= db + dc;
        }
      }
    }
    if (grad) {
      if (faces) {
        if (ok) {
#pragma unroll
          for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) unsafeAtomicAdd(&grad[ax * N + vid[k]], (float)g[k][ax]);
        }
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            float* d = &grad[ax * N + 3 * m + k];
            *d = accumulate ? *d + (float)g[k][ax] : (float)g[k][ax];
          }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = loss;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_equi_loss(const double* __restrict__ partial, int64_t nb, int64_t M,
                                                   float* __restrict__ loss) {
  __shared__ double red[4];
  double sum = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) sum += partial[b];
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) loss[0] = M > 0 ? (float)(((red[0] + red[1]) + (red[2] + red[3])) / (3.0 * (double)M)) : 0.f;
}

__global__ __launch_bounds__(256) void k_zero_f32(float* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.f;
}

int64_t equi_blocks(int64_t n_faces) { return (n_faces + kEquiBlock - 1) / kEquiBlock; }

hipError_t launch_equi(const tsr_scene_dev& sc, float weight, bool accumulate, float* loss, float* grad,
                       double* partial, hipStream_t st) {
  const int64_t M = sc.n_faces, N = sc.n_vertices;
  const int64_t nb = equi_blocks(M);
  if (grad && !accumulate && (sc.faces || N > 3 * M)) {
    // indexed meshes add into the output; soups leave vertices past 3M untouched otherwise
    const int64_t blocks = std::min<int64_t>((3 * N + 255) / 256, 8192);
    if (blocks > 0) TSR_LAUNCH("zero_f32", k_zero_f32, dim3((unsigned)blocks), dim3(256), 0, st, grad, 3 * N);
  }
  const double gscale = M > 0 ? 2.0 * (double)weight / (3.0 * (double)M) : 0.0;
  if (nb > 0)
    TSR_LAUNCH("equi", k_equi, dim3((unsigned)nb), dim3(kEquiBlock), 0, st, sc.pos, N, sc.faces, M, gscale,
               accumulate ? 1 : 0, grad, partial);
  if (loss) TSR_LAUNCH("equi_loss", k_equi_loss, dim3(1), dim3(256), 0, st, partial, nb, M, loss);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- no-allocation variant
// The partial sums of tsr_equilateral_noalloc live in this file-scope device array (one copy per
// GPU, held until the process ends) instead of a caller-provided scratch buffer.  Host code never
// passes the array's name to a kernel: the name is a host-side stand-in, not a device address.
// The device address is looked up once per device with hipGetSymbolAddress and cached.
static __device__ __align__(256) double scratch[kEquiStaticPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t equi_static_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    // the caller made `device` current
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace tsr
