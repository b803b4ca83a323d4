// Internal device-side definitions of the gfx950 rasterizer: per-face record layout, the
// per-call view table, and wave64 primitives.  Included by the .hip sources only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsr.h"

namespace tsr {

constexpr int kTile = TSR_TILE;          // 16x16 pixel tiles
constexpr int kBlock = 256;              // one pixel per lane, 4 waves of 8x8 pixels per tile
constexpr int kWave = 64;

// Per-(view, face) setup record, 24 dwords (96 B), written by the projection kernel for
// visible faces only.  Coordinates are face-local: dx = u - u0, dy = v - v0 with (u0, v0)
// the top-left pixel of the face's pixel rectangle, so per-pixel FP32 math works on small
// exact integers.
//   E_k(p) = a_k dx + b_k dy + c_k = -L_k(p) / r  (eq. 2 edge function over phi(s) = -r)
//   rho(p) = min_k E_k(p) = phi(p) / phi(s)      (eq. 3 before ReLU and exponent)
//   colour_ch(p) = P_ch dx + Q_ch dy + R_ch        (barycentric interpolation is affine in p)
enum RecordField : int {
  kRecEdge = 0,      // [3][3] a_k, b_k, c_k
  kRecCol = 9,       // [3][3] P_ch, Q_ch, R_ch
  kRecOpa = 18,      // o_F
  kRecZ = 19,        // z_F
  kRecU0 = 20,       // u0 as a float (an exact integer)
  kRecV0 = 21,       // v0 as a float (an exact integer)
  kRecU1V1 = 22,     // int u1 | (v1 << 16)  (image sizes are at most 16384)
  kRecSigma = 23,    // the face's window exponent sigma (eq. 3)
  kRecDwords = 24
};
// With perspective-correct interpolation the colour planes hold the numerators N_ch of the
// perspective-correct colour, sum_k lambda_k c_k / z_k, and three dwords the plane of the
// denominator W = sum_k lambda_k / z_k (W = 1 / depth of the face's plane along the ray); the
// depth z_F, the rectangle's end and the per-face exponent are not stored.
enum PerspField : int { kRecWa = kRecZ, kRecWb = kRecU1V1, kRecWc = kRecSigma };

// Per-(view, face) gradient accumulator, 20 values, filled by the backward blend:
// dL/d(a_k, b_k, c_k) for the three edges, dL/d(P, Q, R) per channel, dL/do_F, dL/dz_F.
// Wave partial sums are FP32; they are accumulated across waves and tiles in acc_t.
enum GradField : int { kGEdge = 0, kGCol = 9, kGOpa = 18, kGZ = 19, kGradDwords = 20 };
// Perspective-correct mode: the colour slots hold dL/d(N_ch plane), kGZ dL/d(constant of the W
// plane); the W plane's two slopes go to a second per-(view, face) accumulator of 2 floats.
enum GradPerspField : int { kGWc = kGZ };
#ifndef TSR_ACC_F64
#define TSR_ACC_F64 0
#endif
#if TSR_ACC_F64
typedef double acc_t;
#else
typedef float acc_t;
#endif

struct ViewDesc {
  int32_t width, height, tiles_x, tiles_y;
  int32_t tile_off;        // first global tile id of this view
  int32_t pad;
  int64_t pix_off;         // first packed pixel of this view
  float fx, fy, cx, cy;
};

struct ViewTable {
  ViewDesc v[TSR_MAX_VIEWS];
  int32_t n_views;
  int32_t n_tiles;         // total tiles
  int64_t n_faces;         // M
  int32_t face_sigma;      // the scene has per-face window exponents (records hold each face's)
  int32_t pad;
};

__device__ __forceinline__ int view_of_tile(const ViewTable& vt, int tile) {
  int v = 0;
  for (int i = 1; i < vt.n_views; ++i)
    if (tile >= vt.v[i].tile_off) v = i;
  return v;
}

// ---------------------------------------------------------------------------- wave64 DPP
// Row-wise DPP butterflies, then the legacy gfx9 row broadcasts, leave the wave total in
// lane 63.  Every lane must be active.

#define TSR_DPP(v, ctrl, rmask, bmask)                                                     \
  __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, rmask, bmask, false))

__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += TSR_DPP(v, 0xB1, 0xF, 0xF);     // quad_perm [1,0,3,2]
  v += TSR_DPP(v, 0x4E, 0xF, 0xF);     // quad_perm [2,3,0,1]
  v += TSR_DPP(v, 0x124, 0xF, 0xF);    // row_ror:4
  v += TSR_DPP(v, 0x128, 0xF, 0xF);    // row_ror:8  -> every lane holds its row's sum
  v += TSR_DPP(v, 0x142, 0xA, 0xF);    // row_bcast:15 into rows 1 and 3
  v += TSR_DPP(v, 0x143, 0xC, 0xF);    // row_bcast:31 into rows 2 and 3
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to_lane63(v)), 63));
}

// Wave totals of 20 per-lane values with a transposing butterfly: at each level a pair of
// vectors (x, y) becomes one, the lanes on one side of the level's partner bit keeping x summed
// with their partner lane and the others keeping y.
//   v_permlane32_swap (partner l ^ 32): 20 -> 10 vectors;
//   v_permlane16_swap (rows 0 <-> 1, 2 <-> 3): 10 -> 5; row r now holds value 4 j + {0, 2, 1, 3}[r]
//     of vector j, summed over the four rows;
//   inside each row, bit 3 (partner l ^ 8, row_ror:8): 5 -> 3 (the odd vector is summed over
//     the pair); bit 2 (partner l ^ 7, row_half_mirror): 3 -> 2; bits 1 and 0 (quad_perm):
//     both summed.
// The partners span all 64 lanes, so every kept value is a wave total.  The paired vector's
// totals (16 values) are read on lanes x = 0, 4, 8, 12 of each row, the odd vector's (the other
// 4, the same on every lane of a row) on lane x = 1: the result is value wave_sum20_slot() on
// the 20 lanes where that is not -1.  Every lane must be active.
__device__ __forceinline__ int wave_sum20_slot() {
  const int r = (threadIdx.x & 63) >> 4, x = threadIdx.x & 15;
  const int rmap = r == 0 ? 0 : (r == 1 ? 2 : (r == 2 ? 1 : 3));
  return (x & 3) == 0 ? 4 * (2 * ((x >> 2) & 1) + ((x >> 3) & 1)) + rmap : (x == 1 ? 16 + rmap : -1);
}

// The adds below are kept out of FMA contraction with any product that feeds them: an FMA
// cannot take a DPP operand, a plain add folds the lane exchange into itself.
template <int CTRL>
__device__ __forceinline__ float pair_level(float x, float y, bool bit) {
#pragma clang fp contract(off)
  const float sx = x + TSR_DPP(x, CTRL, 0xF, 0xF);
  const float sy = y + TSR_DPP(y, CTRL, 0xF, 0xF);
  return bit ? sy : sx;
}

__device__ __forceinline__ float wave_sum20(const float* v) {
#pragma clang fp contract(off)
  float s[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * i]), __float_as_uint(v[2 * i + 1]), false,
                                                    false);
    s[i] = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  }
  float t[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(s[2 * j]), __float_as_uint(s[2 * j + 1]), false,
                                                    false);
    t[j] = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  }
  const int x = threadIdx.x & 15;
  const bool b2 = x & 4, b3 = x & 8;
  const float a0 = pair_level<0x128>(t[0], t[1], b3);                  // row_ror:8
  const float a1 = pair_level<0x128>(t[2], t[3], b3);
  float a2 = t[4] + TSR_DPP(t[4], 0x128, 0xF, 0xF);
  float bb = pair_level<0x141>(a0, a1, b2);                            // row_half_mirror
  a2 += TSR_DPP(a2, 0x141, 0xF, 0xF);
  bb += TSR_DPP(bb, 0x4E, 0xF, 0xF);                                   // quad_perm [2,3,0,1]
  a2 += TSR_DPP(a2, 0x4E, 0xF, 0xF);
  bb += TSR_DPP(bb, 0xB1, 0xF, 0xF);                                   // quad_perm [1,0,3,2]
  a2 += TSR_DPP(a2, 0xB1, 0xF, 0xF);
  float out = (x & 3) == 0 ? bb : a2;
  // keeps the sums in this (full-wave) part of the code instead of letting them move into a
  // caller's branch on the slot
  asm volatile("" : "+v"(out));
  return out;
}

// The same butterfly over 24 values: the third permlane16 pair (values 16..23) is split by bit 3
// like the first two and then summed over bits 2..0; its totals are read on lanes x = 1 (bit 3
// clear) and x = 9 (bit 3 set) of each row.  Result: value wave_sum24_slot() on the 24 lanes
// where that is not -1.  Every lane must be active.
__device__ __forceinline__ int wave_sum24_slot() {
  const int r = (threadIdx.x & 63) >> 4, x = threadIdx.x & 15;
  const int rmap = r == 0 ? 0 : (r == 1 ? 2 : (r == 2 ? 1 : 3));
  const int b3 = (x >> 3) & 1;
  if ((x & 3) == 0) return 4 * (2 * ((x >> 2) & 1) + b3) + rmap;
  return (x & 7) == 1 ? 16 + 4 * b3 + rmap : -1;
}

__device__ __forceinline__ float wave_sum24(const float* v) {
#pragma clang fp contract(off)
  float s[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * i]), __float_as_uint(v[2 * i + 1]), false,
                                                    false);
    s[i] = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  }
  float t[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(s[2 * j]), __float_as_uint(s[2 * j + 1]), false,
                                                    false);
    t[j] = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  }
  const int x = threadIdx.x & 15;
  const bool b2 = x & 4, b3 = x & 8;
  const float a0 = pair_level<0x128>(t[0], t[1], b3);                  // row_ror:8
  const float a1 = pair_level<0x128>(t[2], t[3], b3);
  float a2 = pair_level<0x128>(t[4], t[5], b3);
  float bb = pair_level<0x141>(a0, a1, b2);                            // row_half_mirror
  a2 += TSR_DPP(a2, 0x141, 0xF, 0xF);
  bb += TSR_DPP(bb, 0x4E, 0xF, 0xF);                                   // quad_perm [2,3,0,1]
  a2 += TSR_DPP(a2, 0x4E, 0xF, 0xF);
  bb += TSR_DPP(bb, 0xB1, 0xF, 0xF);                                   // quad_perm [1,0,3,2]
  a2 += TSR_DPP(a2, 0xB1, 0xF, 0xF);
  float out = (x & 3) == 0 ? bb : a2;
  asm volatile("" : "+v"(out));
  return out;
}

__device__ __forceinline__ int wave_max_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Wave ballot of a predicate, taken as a lane mask directly (no conversion to an integer first).
__device__ __forceinline__ unsigned long long ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(v, (unsigned)o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

// Exclusive prefix sum of one value per thread over the workgroup (blockDim.x a multiple of
// 64, at most 1024), and the workgroup total.  `wsum` is 16 shared slots.  Every thread of the
// workgroup must call it; it contains two barriers, after which `wsum` may be reused.
__device__ __forceinline__ unsigned long long block_excl_scan_u64(unsigned long long s, unsigned long long* wsum,
                                                                  unsigned long long* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const unsigned long long inc = wave_incl_scan_u64(s);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  unsigned long long before = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    const unsigned long long x = wsum[i];
    if (i < w) before += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return before + inc - s;
}

}  // namespace tsr
