// Internal declarations shared by the kernel sources and the C-ABI layer: the workspace
// layout and the launch sequences.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsr.h"
#include "tsr_device.h"

namespace tsr {

// Device-side copy of the scene pointers (passed by value to kernels).
struct tsr_scene_dev {
  const float* pos;
  const float* col;
  const float* opa;
  const int32_t* faces;
  int64_t n_vertices;
  int64_t n_faces;
  int32_t opa_min;       // face opacity: 0 = vertex mean, 1 = vertex minimum
  const float* face_sigma;   // [M] per-face window exponents, or nullptr (the parameters' sigma)
  float* grad_face_sigma;    // [M] dL/dsigma_m output of the backward, or nullptr
};

// Byte offsets of the workspace regions.  Fixed part first (depends on M, the views and
// their sizes), then the pair buffers (16 B per pair of capacity: sorted pairs + merge temp).
struct WsLayout {
  size_t hdr_k, hdr_overflow;      // int64 K, uint32 overflow flag
  size_t hdr_queue;                // int32 work-queue counter of the persistent training kernel
  size_t hdr_sticky;               // uint32: some binning since the last tsr_check overflowed
  size_t pose_acc;                 // double [kSumCopies][V][6]
  size_t loss_acc;                 // double [kSumCopies][V]
  size_t loss_part;                // float [T][4]: L1 loss of each (tile, 8x8 quadrant)
  size_t counts;                   // uint32 [V*M]
  size_t records;                  // float  [V*M][24]
  size_t grad_acc;                 // float  [V*M][20]
  size_t sig_acc;                  // float  [V*M]: dL/dsigma of each (view, face) (per-face exponents)
  size_t persp_acc;                // float  [V*M][2]: dL/d(W plane slopes) (perspective-correct mode)
  size_t tile_cnt;                 // uint32 [T][4]: [0] faces with <= 4 tiles, [2] larger faces (later
                                   // their emission cursor), [1] and [3] unused, so that every counter
                                   // the atomics hit sits alone in its 8-byte word; then the uint32
                                   // long-tile counter (all filled together)
  size_t long_cnt;                 // uint32: tiles whose list is too long for the register sort
  size_t long_list;                // uint32 [T]: those tiles
  size_t vis_cnt;                  // uint32 [NB]: visible (view, face) pairs of each visible-list segment
  size_t vis_off;                  // uint32 [NB]: exclusive scan of vis_cnt
  size_t vis_total;                // uint32: total visible (view, face) pairs
  size_t vis_list;                 // VisEntry [NB][256]: the visible (view, face) pairs of segment b
                                   // (first vis_cnt[b] entries)
  size_t vis_dense;                // uint32 [V*M]: the same ids, compacted (first vis_total entries)
  size_t ranges;                   // uint32 [T][2]
  size_t order;                    // int32  [T] tile schedule (longest lists first)
  size_t n_last;                   // int32  [P]
  size_t t_last;                   // float  [P]
  size_t fixed_end;
  size_t pairs;                    // uint64 [cap]
  size_t temp;                     // uint64 [cap]
  size_t total;
  int64_t capacity;
};

constexpr int kOrderBuckets = 1024;    // tile-length buckets of the longest-first schedule
constexpr int kSumCopies = 64;         // copies of the FP64 pose / loss sums (workgroup b adds into
                                       // copy b % kSumCopies, so few atomics meet on one address)
constexpr int kProjBlock = 256;        // threads per projection workgroup; entries per visible-list segment

// Pre-test rounds per projection workgroup (kProjBlock pairs each) and the visible-list
// segments that the projection writes: one per workgroup for one round, one per wave for four.
inline int proj_rounds(int n_views) { return n_views == 1 ? 1 : 4; }
inline int64_t proj_segments(int64_t n_pairs, int n_views) {
  const int64_t r = proj_rounds(n_views);
  return r * ((n_pairs + r * kProjBlock - 1) / (r * kProjBlock));
}
constexpr int kRegSortMax = 1024;      // tile lists up to this length are sorted in registers
constexpr int kWaveSortMax = 512;      // ... by one wave (longer ones by a whole workgroup)
constexpr int kSmallTiles = 4;         // faces overlapping at most this many tiles record their slots
constexpr int kTileCntStride = 4;     // dwords per tile in the tile-counter array
constexpr uint32_t kSkipSlot = 0xffffffffu;   // recorded slot of a tile the tight binning leaves out
constexpr int kTileQuads = 4;          // 8x8 quadrants of a 16x16 tile (one blend wave each)
constexpr int kNormalPart = 8;         // floats of normal-loss sums per blend wave (mapping step)

// What the emission of one visible (view, face) pair needs, written by the projection in the
// order of its workgroup's threads: id g = v * M + m, the global id of the first tile of its
// tile rectangle, the rectangle's extent and its view's tile row pitch, the float32 z_F bits of
// its sort key, and (faces over at most kSmallTiles tiles) its slot in each tile, row-major
// over the rectangle.
struct VisEntry {
  uint32_t g, tile0, ext, zbits;   // ext = (tiles wide - 1) | (tiles high - 1) << 10 |
                                   //       (view's tiles_x - 1) << 20 (each at most 1023)
  uint32_t slot[kSmallTiles];
};

constexpr int kOrderInSortMax = 8192;  // tile counts whose longest-first order the binning builds

// Longest-first order of the tiles for the training kernel's queue, by one workgroup: a
// counting sort of the tiles by list length, descending (lengths of kOrderBuckets - 1 and more
// share the first bucket).  `hist` is kOrderBuckets shared counters, `wsum` 16 shared slots;
// blockDim.x divides kOrderBuckets.
__device__ inline void build_tile_order(const uint32_t* __restrict__ ranges, int n_tiles, int* __restrict__ order,
                                 uint32_t* hist, unsigned long long* wsum) {
  const int nb = blockDim.x;
  for (int b = threadIdx.x; b < kOrderBuckets; b += nb) hist[b] = 0u;
  __syncthreads();
  // bucket kOrderBuckets - 1 - length: an ascending scan then places long lists first.  Each
  // thread loads four tiles' ranges before their LDS atomics, so the loads overlap.
  constexpr int kU = 4;
  for (int t0 = threadIdx.x; t0 < n_tiles; t0 += kU * nb) {
    uint32_t len[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * nb;
      len[u] = t < n_tiles ? ranges[2 * t + 1] - ranges[2 * t] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (t0 + u * nb < n_tiles) atomicAdd(&hist[kOrderBuckets - 1 - (int)min(len[u], (uint32_t)kOrderBuckets - 1u)], 1u);
  }
  __syncthreads();
  const int per = kOrderBuckets / nb;
  unsigned long long sum = 0, tot;
  for (int k = 0; k < per; ++k) sum += hist[threadIdx.x * per + k];
  unsigned long long run = block_excl_scan_u64(sum, wsum, &tot);
  for (int k = 0; k < per; ++k) {
    const uint32_t h = hist[threadIdx.x * per + k];
    hist[threadIdx.x * per + k] = (uint32_t)run;
    run += h;
  }
  __syncthreads();
  for (int t0 = threadIdx.x; t0 < n_tiles; t0 += kU * nb) {
    uint32_t len[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * nb;
      len[u] = t < n_tiles ? ranges[2 * t + 1] - ranges[2 * t] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * nb;
      if (t < n_tiles) {
        const uint32_t pos = atomicAdd(&hist[kOrderBuckets - 1 - (int)min(len[u], (uint32_t)kOrderBuckets - 1u)], 1u);
        order[pos] = t;
      }
    }
  }
}

// Training-kernel schedule (chosen by the autotuner; the default is one workgroup per tile).
struct TrainSchedule {
  int persistent;       // 0: one workgroup per tile; 1: persistent workgroups pull tiles from a queue
  int order;            // 0: tile-id order; 1: longest tile lists first
  int grid;             // persistent workgroups (0 = 2048)
};

// Optional per-kernel timing with HIP events recorded on the launch stream (off by default).
// prof_begin returns a token (-1 when profiling is off); prof_end closes it under `name`.
int prof_begin(hipStream_t st);
void prof_end(int token, const char* name, hipStream_t st);

#define TSR_LAUNCH(name, kernel, grid, block, shmem, st, ...)                 \
  do {                                                                        \
    const int tsr_tok_ = ::tsr::prof_begin(st);                               \
    hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__);          \
    ::tsr::prof_end(tsr_tok_, name, st);                                      \
  } while (0)

hipError_t launch_ws_init(char* ws, hipStream_t st);

hipError_t launch_bin(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                      const WsLayout& L, char* ws, bool sort, hipStream_t st);

// Normal channels of the separate forward and backward walks (mapping step, Sec. 3.4): each
// face's world unit normal composited like a colour constant over the face.  face_normal and
// grad are [M][4] floats (x, y, z, 0) per face, summed over the views in grad (which the
// caller zero-fills); map (forward, may be null: N in the camera frame) and target are packed
// like colour; part (forward) holds 8 floats per wave of each tile (kernel-written), count
// (backward) the valid target pixels of each view.
struct NormalChannels {
  const float* face_normal;
  float* map;
  float* grad;
  const float* poses;
  const float* target;
  const uint32_t* count;
  float* part;
  float w_norm;
};

hipError_t launch_forward(const ViewTable& vt, const tsr_params& p, const WsLayout& L, char* ws, float* color,
                          float* depth, float* trans, hipStream_t st, const NormalChannels* nc = nullptr);

hipError_t launch_backward(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                           const WsLayout& L, char* ws, const float* gcolor, const float* gdepth,
                           const float* gtrans, const float* tcolor, const float* tdepth, float* color,
                           float* depth, float* trans, float* loss, float* grad_pos, float* grad_col,
                           float* grad_opa, float* grad_pose, bool fused_train, const TrainSchedule& sched,
                           hipStream_t st, const NormalChannels* nc = nullptr, bool order_built = false);
// (order_built: a forward since the binning, on the same stream, built the longest-first tile
// order the separate backward walks in, so it is not built again.)

// D-SSIM (Sec. 3.4, eq. 8): output tile of the stencil kernels and the window radius.
constexpr int kSsimTW = 32;
constexpr int kSsimTH = 32;
constexpr int kSsimR = 5;               // 11 x 11 window

// Per-view geometry of the D-SSIM kernels (a kernel argument).  Workgroup b works on view v
// with blk_off[v] <= b < blk_off[v + 1]: channel-major, then row-major over the view's tiles.
struct SsimTable {
  int32_t width[TSR_MAX_VIEWS], height[TSR_MAX_VIEWS];
  int32_t tiles_x[TSR_MAX_VIEWS], tiles_y[TSR_MAX_VIEWS];
  int64_t pix_off[TSR_MAX_VIEWS];       // pixels of the views before v
  int32_t blk_off[TSR_MAX_VIEWS + 1];
  int32_t n_views;
  int64_t n_pixels;
  float g[2 * kSsimR + 1];              // normalised 1-D Gaussian factor of the window
};

// Returns 0, or -1 when a view size is outside (0, 16384] or n_views outside [1, TSR_MAX_VIEWS].
int build_ssim_table(const tsr_intrinsics* intr, int n_views, SsimTable* t);
size_t ssim_scratch_bytes(const SsimTable& t);
hipError_t launch_dssim(const SsimTable& t, const float* color, const float* target, float weight,
                        bool accumulate, float* loss, float* grad, char* scratch, hipStream_t st);
// D-SSIM statistics and the colour / depth seeds of the full photometric loss in `scratch`;
// returns the seed pointers (inside scratch) through gcolor / gdepth.
hipError_t launch_photo_seeds(const SsimTable& t, const float* color, const float* target, const float* depth,
                              const float* tdepth, float w_ssim, float w_color, float w_depth, float* loss,
                              char* scratch, float** gcolor, float** gdepth, hipStream_t st);

// Equilateral regulariser (Sec. 3.4, eq. 14): workgroups of one launch over M faces, and the
// launch (loss and/or gradient; `partial` holds one double per workgroup).
int64_t equi_blocks(int64_t n_faces);
// Partials of the allocation-free variant: one double per 256-face workgroup in a static
// device array of this many entries (128 KiB per GPU).
constexpr int64_t kEquiStaticPartials = 16384;
// Device address of that array on `device` (which must be current), looked up on first use.
hipError_t equi_static_scratch(int device, double** out);
hipError_t launch_equi(const tsr_scene_dev& sc, float weight, bool accumulate, float* loss, float* grad,
                       double* partial, hipStream_t st);

// Per-face screen statistics (pruning, densification and keyframing tests of Sec. 3.4).
hipError_t launch_face_area(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                            float* area, hipStream_t st);
hipError_t launch_face_stats(const ViewTable& vt, const tsr_params& p, const WsLayout& L, char* ws,
                             uint32_t* coverage, uint32_t* visible, hipStream_t st);

// Normal supervision (Sec. 3.4): scratch layout of the normal-loss step (byte offsets).
struct NormalScratch {
  size_t col, gcol, nw, seed, depth, zeros, gpos, gopa, gpose, count, acc, total;
};
NormalScratch normal_scratch(int64_t n_vertices, int64_t n_pixels);
hipError_t launch_sensor_normals(const ViewTable& vt, const float* depth, float* normals, hipStream_t st);
hipError_t launch_train_normal(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                               const WsLayout& L, char* ws, const float* target, float w_norm, float* normal_map,
                               float* loss, float* grad_pos, float* grad_opa, float* grad_pose, bool accumulate,
                               char* scratch, int64_t n_pixels, hipStream_t st);

// The full mapping energy on one binning (photometric, depth and normal terms): scratch
// layout after the D-SSIM scratch (byte offsets from the start of the whole scratch).
struct MappingScratch {
  size_t nrm, gacc, part, count, acc, total;
};
MappingScratch mapping_scratch(size_t ssim_bytes, int64_t n_faces, int64_t n_tiles);
hipError_t launch_train_mapping(const tsr_scene_dev& sc, const float* poses, const ViewTable& vt, const tsr_params& p,
                                const WsLayout& L, char* ws, const SsimTable& t, const float* target_color,
                                const float* target_depth, const float* target_normals, float w_ssim, float w_norm,
                                float* color, float* depth, float* trans, float* normal_map, float* loss,
                                float* loss_norm, float* grad_pos, float* grad_col, float* grad_opa,
                                float* grad_pose, char* scratch, hipStream_t st);

hipError_t launch_pose_step(float* poses, const float* grad_pose, int n_views, float lr_t, float lr_r,
                            hipStream_t st);
hipError_t launch_pose_compose(const float* tau, const float* poses, int n_views, float* out, hipStream_t st);
hipError_t launch_pose_tau_grad(const float* tau, const float* grad_pose, int n_views, float* grad_tau,
                                hipStream_t st);

}  // namespace tsr
