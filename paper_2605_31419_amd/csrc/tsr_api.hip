// C ABI of the rasterizer: argument validation, workspace layout, launch sequences and
// error reporting.  Every entry point only enqueues work on the caller's stream except
// tsr_check and tsr_count, which synchronise it.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tsr_internal.h"

// ---------------------------------------------------------------------------- kernel timing
namespace tsr {
namespace {
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
std::map<std::string, std::pair<long long, double>> g_prof_acc;   // name -> (launches, total ms)

hipEvent_t pool_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

int prof_begin(hipStream_t st) {
  if (!g_prof_on) return -1;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfRec r{nullptr, pool_event(), pool_event()};
  if (!r.a || !r.b) return -1;
  (void)hipEventRecord(r.a, st);
  g_prof_pending.push_back(r);
  return (int)g_prof_pending.size() - 1;
}

void prof_end(int token, const char* name, hipStream_t st) {
  if (token < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (token >= (int)g_prof_pending.size()) return;
  g_prof_pending[token].name = name;
  (void)hipEventRecord(g_prof_pending[token].b, st);
}
}  // namespace tsr

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(TSR_EHIP, "%s: %s", where, hipGetErrorString(e));
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

using tsr::ViewTable;
using tsr::WsLayout;

int check_scene(const tsr_scene* sc) {
  if (!sc) return fail(TSR_EINVAL, "scene is NULL");
  if (sc->n_faces < 0 || sc->n_vertices < 0) return fail(TSR_EINVAL, "negative scene size");
  if (sc->n_faces > 0 && (!sc->pos || !sc->col || !sc->opa))
    return fail(TSR_EINVAL, "scene pos/col/opa pointer is NULL");
  if (!sc->faces && sc->n_vertices < 3 * sc->n_faces)
    return fail(TSR_EINVAL, "soup needs n_vertices >= 3 * n_faces (%lld < %lld)", (long long)sc->n_vertices,
                (long long)(3 * sc->n_faces));
  return TSR_OK;
}

int build_views(const tsr_scene* sc, const tsr_intrinsics* intr, int n_views, ViewTable* vt) {
  if (!intr) return fail(TSR_EINVAL, "intrinsics pointer is NULL");
  if (n_views < 1 || n_views > TSR_MAX_VIEWS) return fail(TSR_EINVAL, "n_views = %d outside [1, %d]", n_views, TSR_MAX_VIEWS);
  memset(vt, 0, sizeof *vt);
  int64_t tiles = 0, pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const tsr_intrinsics& c = intr[v];
    if (c.width <= 0 || c.height <= 0 || c.width > 16384 || c.height > 16384)
      return fail(TSR_EINVAL, "view %d: image size %dx%d outside (0, 16384]", v, c.width, c.height);
    tsr::ViewDesc& d = vt->v[v];
    d.width = c.width;
    d.height = c.height;
    d.tiles_x = (c.width + TSR_TILE - 1) / TSR_TILE;
    d.tiles_y = (c.height + TSR_TILE - 1) / TSR_TILE;
    d.tile_off = (int32_t)tiles;
    d.pix_off = pix;
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    tiles += (int64_t)d.tiles_x * d.tiles_y;
    pix += (int64_t)c.width * c.height;
  }
  if (tiles >= (1ll << 31)) return fail(TSR_EINVAL, "too many tiles");
  vt->n_views = n_views;
  vt->n_tiles = (int32_t)tiles;
  vt->n_faces = sc->n_faces;
  vt->face_sigma = sc->face_sigma ? 1 : 0;
  if ((int64_t)n_views * sc->n_faces >= (1ll << 31))
    return fail(TSR_EINVAL, "n_views * n_faces = %lld must be below 2^31", (long long)n_views * sc->n_faces);
  return TSR_OK;
}

int64_t total_pixels(const ViewTable& vt) {
  const tsr::ViewDesc& d = vt.v[vt.n_views - 1];
  return d.pix_off + (int64_t)d.width * d.height;
}

WsLayout layout(const ViewTable& vt, int64_t cap) {
  WsLayout L;
  const int64_t nf = (int64_t)vt.n_views * vt.n_faces;
  const int64_t P = total_pixels(vt);
  size_t o = 0;
  L.hdr_k = 0;
  L.hdr_overflow = 8;
  L.hdr_queue = 12;
  L.hdr_sticky = 16;
  o = 256;
  L.pose_acc = o; o = align_up(o + sizeof(double) * tsr::kSumCopies * 6 * vt.n_views);
  L.loss_acc = o; o = align_up(o + sizeof(double) * tsr::kSumCopies * vt.n_views);
  L.loss_part = o; o = align_up(o + sizeof(float) * 4 * vt.n_tiles);
  L.counts = o; o = align_up(o + sizeof(uint32_t) * nf);
  L.records = o; o = align_up(o + sizeof(float) * tsr::kRecDwords * nf);
  L.grad_acc = o; o = align_up(o + sizeof(tsr::acc_t) * tsr::kGradDwords * nf);
  L.sig_acc = o; o = align_up(o + sizeof(float) * nf);
  L.persp_acc = o; o = align_up(o + sizeof(float) * 2 * nf);
  const int64_t nb = tsr::proj_segments(nf, vt.n_views);
  L.tile_cnt = o;
  L.long_cnt = o + sizeof(uint32_t) * tsr::kTileCntStride * vt.n_tiles;
  o = align_up(o + sizeof(uint32_t) * (tsr::kTileCntStride * vt.n_tiles + 1));
  L.long_list = o; o = align_up(o + sizeof(uint32_t) * vt.n_tiles);
  L.vis_cnt = o; o = align_up(o + sizeof(uint32_t) * nb);
  L.vis_off = o; o = align_up(o + sizeof(uint32_t) * nb);
  L.vis_total = o; o = align_up(o + sizeof(uint32_t));
  L.vis_list = o; o = align_up(o + sizeof(tsr::VisEntry) * nb * tsr::kProjBlock);
  L.vis_dense = o; o = align_up(o + sizeof(uint32_t) * nf);
  L.ranges = o; o = align_up(o + sizeof(uint32_t) * 2 * vt.n_tiles);
  L.order = o; o = align_up(o + sizeof(int32_t) * vt.n_tiles);
  L.n_last = o; o = align_up(o + sizeof(int32_t) * P);
  L.t_last = o; o = align_up(o + sizeof(float) * P);
  L.fixed_end = o;
  L.pairs = o; o = align_up(o + sizeof(uint64_t) * cap);
  L.temp = o; o = align_up(o + sizeof(uint64_t) * cap);
  L.total = o;
  L.capacity = cap;
  return L;
}

// Capacity implied by a workspace of ws_bytes, or an error when it cannot hold the fixed part.
int layout_for(const ViewTable& vt, size_t ws_bytes, WsLayout* L) {
  WsLayout z = layout(vt, 0);
  if (ws_bytes < z.total) return fail(TSR_EWORKSPACE, "workspace of %zu bytes is below the %zu-byte minimum", ws_bytes, z.total);
  int64_t cap = (int64_t)((ws_bytes - z.total) / 16);
  if (cap > (int64_t)0x7fffffff) cap = 0x7fffffff;
  while (cap > 0 && layout(vt, cap).total > ws_bytes) --cap;
  *L = layout(vt, cap);
  return TSR_OK;
}

int check_params(const tsr_params* p) {
  if (!p) return fail(TSR_EINVAL, "params is NULL");
  if (!(p->sigma > 0.f)) return fail(TSR_EINVAL, "sigma must be > 0");
  if (!(p->t_min >= 0.f && p->t_min < 1.f)) return fail(TSR_EINVAL, "t_min must be in [0, 1)");
  if (!(p->r_min >= 0.f) || !(p->z_near == p->z_near)) return fail(TSR_EINVAL, "bad r_min / z_near");
  if (p->opacity_min != 0 && p->opacity_min != 1) return fail(TSR_EINVAL, "opacity_min must be 0 or 1");
  if (p->tight_tiles != 0 && p->tight_tiles != 1) return fail(TSR_EINVAL, "tight_tiles must be 0 or 1");
  if (p->perspective != 0 && p->perspective != 1) return fail(TSR_EINVAL, "perspective must be 0 or 1");
  return TSR_OK;
}

tsr::tsr_scene_dev dev_scene(const tsr_scene* sc, const tsr_params* p = nullptr) {
  tsr::tsr_scene_dev d;
  d.opa_min = p ? p->opacity_min : 0;
  d.pos = sc->pos;
  d.col = sc->col;
  d.opa = sc->opa;
  d.faces = sc->faces;
  d.n_vertices = sc->n_vertices;
  d.n_faces = sc->n_faces;
  d.face_sigma = sc->face_sigma;
  d.grad_face_sigma = sc->grad_face_sigma;
  return d;
}

// Arguments of the E_equi entry points: positions and faces only (colours and opacities may be
// NULL there).
int check_equi_args(const tsr_scene* scene, const float* loss, const float* grad_pos) {
  if (!scene) return fail(TSR_EINVAL, "scene is NULL");
  if (scene->n_faces < 0 || scene->n_vertices < 0) return fail(TSR_EINVAL, "negative scene size");
  if (scene->n_faces > 0 && !scene->pos) return fail(TSR_EINVAL, "scene pos pointer is NULL");
  if (!scene->faces && scene->n_vertices < 3 * scene->n_faces)
    return fail(TSR_EINVAL, "soup needs n_vertices >= 3 * n_faces (%lld < %lld)", (long long)scene->n_vertices,
                (long long)(3 * scene->n_faces));
  if (!loss && !grad_pos) return fail(TSR_EINVAL, "loss and grad_pos are both NULL");
  return TSR_OK;
}

// Common argument checks of the per-call entry points.
int prepare(const tsr_scene* sc, const float* poses, const tsr_intrinsics* intr, int n_views, const tsr_params* p,
            void* ws, size_t ws_bytes, ViewTable* vt, WsLayout* L) {
  int rc;
  if ((rc = check_scene(sc))) return rc;
  if ((rc = check_params(p))) return rc;
  if (p->perspective && sc->face_sigma)
    return fail(TSR_EINVAL, "perspective-correct interpolation cannot be combined with per-face exponents");
  if (!poses) return fail(TSR_EINVAL, "poses is NULL");
  if (!ws) return fail(TSR_EINVAL, "workspace is NULL");
  if ((rc = build_views(sc, intr, n_views, vt))) return rc;
  return layout_for(*vt, ws_bytes, L);
}

}  // namespace

extern "C" {

const char* tsr_last_error(void) { return g_err.c_str(); }

int tsr_workspace_size(const tsr_scene* scene, const tsr_intrinsics* intr, int n_views, int64_t pair_capacity,
                       size_t* bytes) {
  int rc;
  if ((rc = check_scene(scene))) return rc;
  if (!bytes) return fail(TSR_EINVAL, "bytes is NULL");
  if (pair_capacity < 0 || pair_capacity > 0x7fffffff) return fail(TSR_EINVAL, "pair_capacity outside [0, 2^31)");
  ViewTable vt;
  if ((rc = build_views(scene, intr, n_views, &vt))) return rc;
  *bytes = layout(vt, pair_capacity).total;
  return TSR_OK;
}

int tsr_workspace_init(void* ws, size_t ws_bytes, void* stream) {
  if (!ws) return fail(TSR_EINVAL, "workspace is NULL");
  if (ws_bytes < 256) return fail(TSR_EWORKSPACE, "workspace of %zu bytes is below the 256-byte header", ws_bytes);
  hipError_t e = tsr::launch_ws_init(static_cast<char*>(ws), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_workspace_init launch");
}

int tsr_bin_and_sort(const tsr_scene* scene, const float* poses, const tsr_intrinsics* intr, int n_views,
                     const tsr_params* params, void* ws, size_t ws_bytes, void* stream) {
  ViewTable vt;
  WsLayout L;
  int rc = prepare(scene, poses, intr, n_views, params, ws, ws_bytes, &vt, &L);
  if (rc) return rc;
  hipError_t e = tsr::launch_bin(dev_scene(scene, params), poses, vt, *params, L, static_cast<char*>(ws), true,
                                 static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_bin_and_sort launch");
}

int tsr_count(const tsr_scene* scene, const float* poses, const tsr_intrinsics* intr, int n_views,
              const tsr_params* params, void* ws, size_t ws_bytes, void* stream, int64_t* n_pairs) {
  ViewTable vt;
  WsLayout L;
  int rc = prepare(scene, poses, intr, n_views, params, ws, ws_bytes, &vt, &L);
  if (rc) return rc;
  if (!n_pairs) return fail(TSR_EINVAL, "n_pairs is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = tsr::launch_bin(dev_scene(scene, params), poses, vt, *params, L, static_cast<char*>(ws), false, st);
  if (e != hipSuccess) return hip_fail(e, "tsr_count launch");
  if ((e = hipMemcpyAsync(n_pairs, static_cast<char*>(ws) + L.hdr_k, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(e, "tsr_count copy");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "tsr_count sync");
  return TSR_OK;
}

int tsr_binning_view(const tsr_scene* scene, const tsr_intrinsics* intr, int n_views, const void* ws,
                     size_t ws_bytes, tsr_binning* out) {
  int rc;
  if ((rc = check_scene(scene))) return rc;
  if (!ws || !out) return fail(TSR_EINVAL, "workspace or out is NULL");
  ViewTable vt;
  WsLayout L;
  if ((rc = build_views(scene, intr, n_views, &vt))) return rc;
  if ((rc = layout_for(vt, ws_bytes, &L))) return rc;
  const char* b = static_cast<const char*>(ws);
  out->pairs = reinterpret_cast<const uint64_t*>(b + L.pairs);
  out->ranges = reinterpret_cast<const uint32_t*>(b + L.ranges);
  out->n_pairs = reinterpret_cast<const int64_t*>(b + L.hdr_k);
  out->overflow = reinterpret_cast<const uint32_t*>(b + L.hdr_overflow);
  out->tile_counts = reinterpret_cast<const uint32_t*>(b + L.counts);
  out->records = reinterpret_cast<const float*>(b + L.records);
  out->capacity = L.capacity;
  out->n_tiles = vt.n_tiles;
  out->n_pixels = total_pixels(vt);
  out->last_face = reinterpret_cast<const int32_t*>(b + L.n_last);
  return TSR_OK;
}

int tsr_render_forward(const tsr_scene* scene, const float* poses, const tsr_intrinsics* intr, int n_views,
                       const tsr_params* params, void* ws, size_t ws_bytes, float* color, float* depth, float* trans,
                       void* stream) {
  ViewTable vt;
  WsLayout L;
  int rc = prepare(scene, poses, intr, n_views, params, ws, ws_bytes, &vt, &L);
  if (rc) return rc;
  if (!color || !depth) return fail(TSR_EINVAL, "color or depth output is NULL");
  hipError_t e = tsr::launch_forward(vt, *params, L, static_cast<char*>(ws), color, depth, trans,
                                     static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_render_forward launch");
}

int tsr_render_backward(const tsr_scene* scene, const float* poses, const tsr_intrinsics* intr, int n_views,
                        const tsr_params* params, void* ws, size_t ws_bytes, const float* grad_color,
                        const float* grad_depth, const float* grad_trans, float* grad_pos, float* grad_col,
                        float* grad_opa, float* grad_pose, void* stream) {
  ViewTable vt;
  WsLayout L;
  int rc = prepare(scene, poses, intr, n_views, params, ws, ws_bytes, &vt, &L);
  if (rc) return rc;
  if (!grad_color || !grad_depth) return fail(TSR_EINVAL, "grad_color or grad_depth is NULL");
  tsr::TrainSchedule sched{0, 0, 0};
  hipError_t e = tsr::launch_backward(dev_scene(scene, params), poses, vt, *params, L, static_cast<char*>(ws), grad_color,
                                      grad_depth, grad_trans, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                      grad_pos, grad_col, grad_opa, grad_pose, false, sched,
                                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_render_backward launch");
}

int tsr_render_train_l1(const tsr_scene* scene, const float* poses, const tsr_intrinsics* intr, int n_views,
                        const tsr_params* params, void* ws, size_t ws_bytes, const float* target_color,
                        const float* target_depth, float* color, float* depth, float* trans, float* loss,
                        float* grad_pos, float* grad_col, float* grad_opa, float* grad_pose,
                        const tsr_schedule* schedule, void* stream) {
  ViewTable vt;
  WsLayout L;
  int rc = prepare(scene, poses, intr, n_views, params, ws, ws_bytes, &vt, &L);
  if (rc) return rc;
  if (!target_color || !target_depth) return fail(TSR_EINVAL, "target_color or target_depth is NULL");
  tsr::TrainSchedule sched{0, 0, 0};
  if (schedule) {
    if (schedule->persistent < 0 || schedule->persistent > 1 || schedule->order < 0 || schedule->order > 1 ||
        schedule->grid < 0 || schedule->grid > (1 << 20))
      return fail(TSR_EINVAL, "bad schedule");
    sched = {schedule->persistent, schedule->order, schedule->grid};
  }
  hipError_t e = tsr::launch_backward(dev_scene(scene, params), poses, vt, *params, L, static_cast<char*>(ws), nullptr,
                                      nullptr, nullptr, target_color, target_depth, color, depth, trans, loss,
                                      grad_pos, grad_col, grad_opa, grad_pose, true, sched,
                                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_render_train_l1 launch");
}

int tsr_pose_step(float* poses, const float* grad_pose, int n_views, float lr_trans, float lr_rot, void* stream) {
  if (!poses || !grad_pose) return fail(TSR_EINVAL, "poses or grad_pose is NULL");
  if (n_views < 1 || n_views > TSR_MAX_VIEWS) return fail(TSR_EINVAL, "n_views = %d outside [1, %d]", n_views, TSR_MAX_VIEWS);
  hipError_t e = tsr::launch_pose_step(poses, grad_pose, n_views, lr_trans, lr_rot, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_pose_step launch");
}

int tsr_pose_compose(const float* tau, const float* poses, int n_views, float* out_poses, void* stream) {
  if (!tau || !poses || !out_poses) return fail(TSR_EINVAL, "tau, poses or out_poses is NULL");
  if (n_views < 1 || n_views > TSR_MAX_VIEWS) return fail(TSR_EINVAL, "n_views = %d outside [1, %d]", n_views, TSR_MAX_VIEWS);
  hipError_t e = tsr::launch_pose_compose(tau, poses, n_views, out_poses, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_pose_compose launch");
}

int tsr_pose_tau_grad(const float* tau, const float* grad_pose, int n_views, float* grad_tau, void* stream) {
  if (!tau || !grad_pose || !grad_tau) return fail(TSR_EINVAL, "tau, grad_pose or grad_tau is NULL");
  if (n_views < 1 || n_views > TSR_MAX_VIEWS) return fail(TSR_EINVAL, "n_views = %d outside [1, %d]", n_views, TSR_MAX_VIEWS);
  hipError_t e = tsr::launch_pose_tau_grad(tau, grad_pose, n_views, grad_tau, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_pose_tau_grad launch");
}

int tsr_dssim_scratch_size(const tsr_intrinsics* intr, int n_views, size_t* bytes) {
  if (!bytes) return fail(TSR_EINVAL, "bytes is NULL");
  tsr::SsimTable t;
  if (!intr || tsr::build_ssim_table(intr, n_views, &t) != 0)
    return fail(TSR_EINVAL, "D-SSIM views: need 1 <= n_views <= %d and image sizes in (0, 16384]", TSR_MAX_VIEWS);
  *bytes = tsr::ssim_scratch_bytes(t);
  return TSR_OK;
}

int tsr_dssim(const tsr_intrinsics* intr, int n_views, const float* color, const float* target, float weight,
              int accumulate, float* loss, float* grad_color, void* scratch, size_t scratch_bytes, void* stream) {
  tsr::SsimTable t;
  if (!intr || tsr::build_ssim_table(intr, n_views, &t) != 0)
    return fail(TSR_EINVAL, "D-SSIM views: need 1 <= n_views <= %d and image sizes in (0, 16384]", TSR_MAX_VIEWS);
  if (!color || !target) return fail(TSR_EINVAL, "color or target is NULL");
  if (!loss && !grad_color) return fail(TSR_EINVAL, "loss and grad_color are both NULL");
  if (!scratch) return fail(TSR_EINVAL, "scratch is NULL");
  const size_t need = tsr::ssim_scratch_bytes(t);
  if (scratch_bytes < need) return fail(TSR_EWORKSPACE, "D-SSIM scratch of %zu bytes is below the %zu needed", scratch_bytes, need);
  if (reinterpret_cast<uintptr_t>(scratch) & 255) return fail(TSR_EINVAL, "scratch must be 256-byte aligned");
  hipError_t e = tsr::launch_dssim(t, color, target, weight, accumulate != 0, loss, grad_color,
                                   static_cast<char*>(scratch), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_dssim launch");
}

int tsr_render_train_photometric(const tsr_scene* scene, const float* poses, const tsr_intrinsics* intr, int n_views,
                                 const tsr_params* params, void* ws, size_t ws_bytes, const float* target_color,
                                 const float* target_depth, float w_ssim, float* color, float* depth, float* trans,
                                 float* loss, float* grad_pos, float* grad_col, float* grad_opa, float* grad_pose,
                                 void* scratch, size_t scratch_bytes, void* stream) {
  ViewTable vt;
  WsLayout L;
  int rc = prepare(scene, poses, intr, n_views, params, ws, ws_bytes, &vt, &L);
  if (rc) return rc;
  if (!target_color || !target_depth) return fail(TSR_EINVAL, "target_color or target_depth is NULL");
  if (!color || !depth) return fail(TSR_EINVAL, "color or depth output is NULL (the D-SSIM term reads them)");
  tsr::SsimTable t;
  if (tsr::build_ssim_table(intr, n_views, &t) != 0) return fail(TSR_EINVAL, "bad D-SSIM view table");
  if (!scratch) return fail(TSR_EINVAL, "scratch is NULL");
  const size_t need = tsr::ssim_scratch_bytes(t);
  if (scratch_bytes < need) return fail(TSR_EWORKSPACE, "D-SSIM scratch of %zu bytes is below the %zu needed", scratch_bytes, need);
  if (reinterpret_cast<uintptr_t>(scratch) & 255) return fail(TSR_EINVAL, "scratch must be 256-byte aligned");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  hipError_t e = tsr::launch_forward(vt, *params, L, w, color, depth, trans, st);
  if (e != hipSuccess) return hip_fail(e, "tsr_render_train_photometric forward");
  float *gc = nullptr, *gd = nullptr;
  e = tsr::launch_photo_seeds(t, color, target_color, depth, target_depth, w_ssim, params->w_color, params->w_depth,
                              loss, static_cast<char*>(scratch), &gc, &gd, st);
  if (e != hipSuccess) return hip_fail(e, "tsr_render_train_photometric seeds");
  tsr::TrainSchedule sched{0, 0, 0};
  e = tsr::launch_backward(dev_scene(scene, params), poses, vt, *params, L, w, gc, gd, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, grad_pos, grad_col, grad_opa, grad_pose, false, sched, st, nullptr,
                           true);
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_render_train_photometric backward");
}

int tsr_equilateral_scratch_size(int64_t n_faces, size_t* bytes) {
  if (!bytes) return fail(TSR_EINVAL, "bytes is NULL");
  if (n_faces < 0) return fail(TSR_EINVAL, "negative n_faces");
  *bytes = align_up(sizeof(double) * (size_t)std::max<int64_t>(1, tsr::equi_blocks(n_faces)));
  return TSR_OK;
}

int tsr_equilateral(const tsr_scene* scene, float weight, int accumulate, float* loss, float* grad_pos,
                    void* scratch, size_t scratch_bytes, void* stream) {
  int rc = check_equi_args(scene, loss, grad_pos);
  if (rc) return rc;
  if (!scratch) return fail(TSR_EINVAL, "scratch is NULL");
  const int64_t nb = tsr::equi_blocks(scene->n_faces);
  if (nb > 0x7fffffff) return fail(TSR_EINVAL, "too many faces");
  const size_t need = sizeof(double) * (size_t)std::max<int64_t>(1, nb);
  if (scratch_bytes < need) return fail(TSR_EWORKSPACE, "E_equi scratch of %zu bytes is below the %zu needed", scratch_bytes, need);
  if (reinterpret_cast<uintptr_t>(scratch) & 7) return fail(TSR_EINVAL, "scratch must be 8-byte aligned");
  hipError_t e = tsr::launch_equi(dev_scene(scene), weight, accumulate != 0, loss, grad_pos,
                                  static_cast<double*>(scratch), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_equilateral launch");
}

int tsr_equilateral_noalloc(const tsr_scene* scene, float weight, int accumulate, float* loss, float* grad_pos,
                            void* stream) {
  int rc = check_equi_args(scene, loss, grad_pos);
  if (rc) return rc;
  const int64_t nb = tsr::equi_blocks(scene->n_faces);
  if (nb > tsr::kEquiStaticPartials)
    return fail(TSR_EINVAL, "tsr_equilateral_noalloc takes at most %d faces (got %lld)", TSR_EQUI_NOALLOC_MAX_FACES,
                (long long)scene->n_faces);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "tsr_equilateral_noalloc current device");
  if (st) {
    int sdev = 0;
    if ((e = hipStreamGetDevice(st, &sdev)) != hipSuccess) return hip_fail(e, "tsr_equilateral_noalloc stream device");
    if (sdev != dev) return fail(TSR_EINVAL, "stream belongs to device %d, the current device is %d", sdev, dev);
  }
  double* partial = nullptr;
  if ((e = tsr::equi_static_scratch(dev, &partial)) != hipSuccess)
    return hip_fail(e, "tsr_equilateral_noalloc static scratch address");
  e = tsr::launch_equi(dev_scene(scene), weight, accumulate != 0, loss, grad_pos, partial, st);
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_equilateral_noalloc launch");
}

int tsr_face_stats(const tsr_scene* scene, const float* poses, const tsr_intrinsics* intr, int n_views,
                   const tsr_params* params, void* ws, size_t ws_bytes, float* area, uint32_t* coverage,
                   uint32_t* visible, void* stream) {
  ViewTable vt;
  WsLayout L;
  int rc = prepare(scene, poses, intr, n_views, params, ws, ws_bytes, &vt, &L);
  if (rc) return rc;
  if (!area && !coverage && !visible) return fail(TSR_EINVAL, "area, coverage and visible are all NULL");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (area) e = tsr::launch_face_area(dev_scene(scene, params), poses, vt, *params, area, st);
  if (e == hipSuccess && (coverage || visible))
    e = tsr::launch_face_stats(vt, *params, L, static_cast<char*>(ws), coverage, visible, st);
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_face_stats launch");
}

int tsr_sensor_normals(const float* depth, const tsr_intrinsics* intr, int n_views, float* normals, void* stream) {
  if (!depth || !normals) return fail(TSR_EINVAL, "depth or normals is NULL");
  if (!intr) return fail(TSR_EINVAL, "intrinsics pointer is NULL");
  if (n_views < 1 || n_views > TSR_MAX_VIEWS) return fail(TSR_EINVAL, "n_views = %d outside [1, %d]", n_views, TSR_MAX_VIEWS);
  ViewTable vt;
  memset(&vt, 0, sizeof vt);
  int64_t pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const tsr_intrinsics& c = intr[v];
    if (c.width <= 0 || c.height <= 0 || c.width > 16384 || c.height > 16384)
      return fail(TSR_EINVAL, "view %d: image size %dx%d outside (0, 16384]", v, c.width, c.height);
    if (!(c.fx != 0.f) || !(c.fy != 0.f)) return fail(TSR_EINVAL, "view %d: zero focal length", v);
    vt.v[v].width = c.width;
    vt.v[v].height = c.height;
    vt.v[v].pix_off = pix;
    vt.v[v].fx = c.fx; vt.v[v].fy = c.fy; vt.v[v].cx = c.cx; vt.v[v].cy = c.cy;
    pix += (int64_t)c.width * c.height;
  }
  vt.n_views = n_views;
  hipError_t e = tsr::launch_sensor_normals(vt, depth, normals, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_sensor_normals launch");
}

int tsr_normal_scratch_size(const tsr_scene* scene, const tsr_intrinsics* intr, int n_views, size_t* bytes) {
  int rc;
  if ((rc = check_scene(scene))) return rc;
  if (!bytes) return fail(TSR_EINVAL, "bytes is NULL");
  ViewTable vt;
  if ((rc = build_views(scene, intr, n_views, &vt))) return rc;
  *bytes = tsr::normal_scratch(scene->n_vertices, total_pixels(vt)).total;
  return TSR_OK;
}

int tsr_render_train_normal(const tsr_scene* scene, const float* poses, const tsr_intrinsics* intr, int n_views,
                            const tsr_params* params, void* ws, size_t ws_bytes, const float* target_normals,
                            float w_norm, float* normal_map, float* loss, float* grad_pos, float* grad_opa,
                            float* grad_pose, int accumulate, void* scratch, size_t scratch_bytes, void* stream) {
  ViewTable vt;
  WsLayout L;
  int rc = prepare(scene, poses, intr, n_views, params, ws, ws_bytes, &vt, &L);
  if (rc) return rc;
  if (scene->faces) return fail(TSR_EINVAL, "the normal loss needs a soup (faces == NULL)");
  if (!target_normals) return fail(TSR_EINVAL, "target_normals is NULL");
  if (!scratch) return fail(TSR_EINVAL, "scratch is NULL");
  const int64_t P = total_pixels(vt);
  const size_t need = tsr::normal_scratch(scene->n_vertices, P).total;
  if (scratch_bytes < need) return fail(TSR_EWORKSPACE, "normal-loss scratch of %zu bytes is below the %zu needed", scratch_bytes, need);
  if (reinterpret_cast<uintptr_t>(scratch) & 255) return fail(TSR_EINVAL, "scratch must be 256-byte aligned");
  hipError_t e = tsr::launch_train_normal(dev_scene(scene, params), poses, vt, *params, L, static_cast<char*>(ws),
                                          target_normals, w_norm, normal_map, loss, grad_pos, grad_opa, grad_pose,
                                          accumulate != 0, static_cast<char*>(scratch), P,
                                          static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_render_train_normal launch");
}

int tsr_mapping_scratch_size(const tsr_scene* scene, const tsr_intrinsics* intr, int n_views, size_t* bytes) {
  int rc;
  if ((rc = check_scene(scene))) return rc;
  if (!bytes) return fail(TSR_EINVAL, "bytes is NULL");
  tsr::SsimTable t;
  if (!intr || tsr::build_ssim_table(intr, n_views, &t) != 0)
    return fail(TSR_EINVAL, "views: need 1 <= n_views <= %d and image sizes in (0, 16384]", TSR_MAX_VIEWS);
  ViewTable vt;
  if ((rc = build_views(scene, intr, n_views, &vt))) return rc;
  *bytes = tsr::mapping_scratch(tsr::ssim_scratch_bytes(t), scene->n_faces, vt.n_tiles).total;
  return TSR_OK;
}

int tsr_render_train_mapping(const tsr_scene* scene, const float* poses, const tsr_intrinsics* intr, int n_views,
                             const tsr_params* params, void* ws, size_t ws_bytes, const float* target_color,
                             const float* target_depth, const float* target_normals, float w_ssim, float w_norm,
                             float* color, float* depth, float* trans, float* normal_map, float* loss,
                             float* loss_norm, float* grad_pos, float* grad_col, float* grad_opa, float* grad_pose,
                             void* scratch, size_t scratch_bytes, void* stream) {
  ViewTable vt;
  WsLayout L;
  int rc = prepare(scene, poses, intr, n_views, params, ws, ws_bytes, &vt, &L);
  if (rc) return rc;
  if (scene->faces) return fail(TSR_EINVAL, "the mapping step needs a soup (faces == NULL)");
  if (!target_color || !target_depth || !target_normals)
    return fail(TSR_EINVAL, "target_color, target_depth or target_normals is NULL");
  if (!color || !depth) return fail(TSR_EINVAL, "color or depth output is NULL (the D-SSIM term reads them)");
  tsr::SsimTable t;
  if (tsr::build_ssim_table(intr, n_views, &t) != 0) return fail(TSR_EINVAL, "bad D-SSIM view table");
  if (!scratch) return fail(TSR_EINVAL, "scratch is NULL");
  const size_t need = tsr::mapping_scratch(tsr::ssim_scratch_bytes(t), scene->n_faces, vt.n_tiles).total;
  if (scratch_bytes < need) return fail(TSR_EWORKSPACE, "mapping scratch of %zu bytes is below the %zu needed", scratch_bytes, need);
  if (reinterpret_cast<uintptr_t>(scratch) & 255) return fail(TSR_EINVAL, "scratch must be 256-byte aligned");
  hipError_t e = tsr::launch_train_mapping(dev_scene(scene, params), poses, vt, *params, L, static_cast<char*>(ws), t,
                                           target_color, target_depth, target_normals, w_ssim, w_norm, color, depth,
                                           trans, normal_map, loss, loss_norm, grad_pos, grad_col, grad_opa, grad_pose,
                                           static_cast<char*>(scratch), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TSR_OK : hip_fail(e, "tsr_render_train_mapping launch");
}

int tsr_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(tsr::g_prof_mu);
  tsr::g_prof_on = on != 0;
  return TSR_OK;
}

int tsr_profile_reset(void) {
  std::lock_guard<std::mutex> lk(tsr::g_prof_mu);
  for (auto& r : tsr::g_prof_pending) {
    (void)hipEventSynchronize(r.b);
    tsr::g_prof_pool.push_back(r.a);
    tsr::g_prof_pool.push_back(r.b);
  }
  tsr::g_prof_pending.clear();
  tsr::g_prof_acc.clear();
  return TSR_OK;
}

int tsr_profile_read(char* buf, size_t len) {
  if (!buf || len == 0) return fail(TSR_EINVAL, "profile buffer is NULL");
  std::lock_guard<std::mutex> lk(tsr::g_prof_mu);
  for (auto& r : tsr::g_prof_pending) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return hip_fail(e, "tsr_profile_read sync");
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, r.a, r.b)) != hipSuccess) return hip_fail(e, "tsr_profile_read elapsed");
    auto& acc = tsr::g_prof_acc[r.name ? r.name : "?"];
    acc.first += 1;
    acc.second += (double)ms;
    tsr::g_prof_pool.push_back(r.a);
    tsr::g_prof_pool.push_back(r.b);
  }
  tsr::g_prof_pending.clear();
  std::string out = "{";
  bool first = true;
  for (auto& kv : tsr::g_prof_acc) {
    char item[256];
    snprintf(item, sizeof item, "%s\"%s\": [%lld, %.9g]", first ? "" : ", ", kv.first.c_str(), kv.second.first,
             kv.second.second);
    out += item;
    first = false;
  }
  out += "}";
  if (out.size() + 1 > len) return fail(TSR_EINVAL, "profile buffer too small (%zu bytes needed)", out.size() + 1);
  memcpy(buf, out.c_str(), out.size() + 1);
  return TSR_OK;
}

int tsr_check(const void* ws, void* stream, int64_t* n_pairs) {
  if (!ws) return fail(TSR_EINVAL, "workspace is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  struct {
    int64_t k;
    uint32_t overflow;
    uint32_t queue;
    uint32_t sticky;
    uint32_t pad;
  } h;
  hipError_t e = hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "tsr_check copy");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "tsr_check sync");
  if (n_pairs) *n_pairs = h.k;
  if (h.sticky) {
    // clear the sticky flag (synchronous: tsr_check is never part of a captured graph)
    if ((e = hipMemsetAsync(static_cast<char*>(const_cast<void*>(ws)) + 16, 0, 4, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "tsr_check clear");
  }
  if (h.sticky & 2u) return fail(TSR_EINTERNAL, "a binning found a tile slot outside its tile's range");
  if (h.overflow || h.sticky)
    return fail(TSR_ECAPACITY, "a binning produced more pairs than the workspace capacity (last K = %lld)", (long long)h.k);
  return TSR_OK;
}

}  // extern "C"
