// Host side of the MI355X LM bundle-adjustment library: the C ABI of include/ba.h, device
// memory ownership, observation sorting, the extraction fixpoint driver, the LM loop and the
// PCG driver. Every per-observation step runs in the kernels of ba_kernels.hip.
#include "ba.h"
#include "ba_kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

using namespace iba;

namespace {

struct BaError {
  ba_status code;
  std::string msg;
};

thread_local std::string g_create_error;

#define HIP_CHECK(expr)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw BaError{BA_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)};     \
  } while (0)

#define HIP_LAUNCH_CHECK()                                                                 \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess)                                                                  \
      throw BaError{BA_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)}; \
  } while (0)

// Device allocations of one lifetime group, released together.
struct Arena {
  std::vector<void*> ptrs;
  int64_t bytes = 0;
  template <typename T>
  T* alloc(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw BaError{BA_ERR_OOM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed"};
    }
    ptrs.push_back(p);
    bytes += int64_t(n * sizeof(T));
    return static_cast<T*>(p);
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
};

struct KStat {
  std::string name;
  int64_t launches = 0;
  double ms = 0.0;
  double bytes = 0.0;
};

struct Pending {
  int kid;
  hipEvent_t a, b;
  double bytes;
  int pcg_iter;   // -1 outside the PCG loop
};

// Size limits: the kernels index per-entity arrays with 32-bit products. The largest are
// 16 lanes per point (thread indices up to 16 P) and 3 values per observation (up to 3 N),
// so P and C stay below 2^27 and N below 2^29; every such product then fits in an int.
constexpr int32_t kMaxCams = (int32_t(1) << 27) - 1;
constexpr int32_t kMaxPoints = (int32_t(1) << 27) - 1;
constexpr int64_t kMaxObs = (int64_t(1) << 29) - 1;

// ------------------------------------------------------------------ static scratch
// Scratch of ba_lm_step_noalloc: the per-step buffers of an LM step (fixpoint and damping
// flags, PCG states, reduction partials, camera-pass partials and terms, item tables, the scan
// workspace) live in this array instead of the context's own buffers. Every GPU the library
// runs on holds one copy from the moment the code object loads until the process ends; its
// device address is looked up once per device (scratch_address, from ba_create with that
// device current) and only that address is handed to kernels and copies.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of the scratch array on device dev, which must be current (looked up on the
// first call per device and kept).
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_addr[dev] = p;
  }
  return g_scratch_addr[dev];
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct ba_ctx {
  ba_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int C = 0, P = 0;
  int64_t N = 0;
  std::string err;

  Arena par, obs;
  // parameters: cameras in caller order, points in internal order
  double *d_cams = nullptr, *d_intr = nullptr, *d_pts = nullptr;
  uint8_t* d_fixed = nullptr;
  Cam<double>* d_camd = nullptr;
  Cam<float>* d_camf = nullptr;
  Cam<double>* d_cand_tab = nullptr;
  double* d_cand_cams = nullptr;
  std::vector<int32_t> pt_user;      // internal -> caller point index
  std::vector<int32_t> pt_internal;  // caller -> internal
  std::vector<uint8_t> fixed_h;
  int n_fixed = 0;
  int* d_fixed_rank = nullptr;       // rank of each fixed camera among the fixed ones

  // observations (point-major, full)
  bool have_obs = false, have_priors = false;
  double lam_d = 0.0;
  int *pm_cam = nullptr, *pm_pt = nullptr, *pm_orig = nullptr, *pt_off = nullptr;
  int *cm_off = nullptr, *pt_user_d = nullptr;
  int *inv_cm = nullptr;   // point-major position -> position in the camera-major order
  int *cm_cam = nullptr;   // camera of each camera-major position
  float2* pm_xy = nullptr;
  float* pm_depth = nullptr;
  std::vector<int32_t> pm_orig_h;  // point-major position -> caller observation index

  // extraction
  uint8_t *vrow = nullptr, *vrow_cm = nullptr, *act_c = nullptr, *act_p = nullptr;
  int *rank_c = nullptr, *rank_p = nullptr, *pos_pm = nullptr, *pos_cm = nullptr;
  void* scan_temp = nullptr;                   // device-wide scan workspace
  size_t scan_temp_size = 0;
  int* flags = nullptr;                        // flags[0] changed, flags[1] bad damping
  int *cam_hat = nullptr, *orig_hat = nullptr, *off_hat = nullptr, *pt_src = nullptr;
  int *cam_src = nullptr, *slot_all = nullptr, *cm_off_hat = nullptr, *cm_pt = nullptr,
      *pm_cm = nullptr;
  Cam<double>* camd_hat = nullptr;
  Cam<float>* camf_hat = nullptr;
  float2* xy_hat = nullptr;
  float* depth_hat = nullptr;
  double* Xd = nullptr;
  float* Xf = nullptr;

  // precision-typed buffers (float in MIXED, double in FP64)
  void *cm_e = nullptr, *prec = nullptr;
  void *ce = nullptr, *cm_ce = nullptr;   // rho' e per observation (full-Hessian adjoint)
  bool ce_on = false;                     // set while the full-Hessian adjoint runs
  void *w = nullptr, *eh = nullptr, *xcw = nullptr, *pm_xcw = nullptr, *cm_eh = nullptr,
       *V = nullptr, *Vinv = nullptr, *zq = nullptr, *Ustar = nullptr, *mvt = nullptr;
  double *gp = nullptr, *hp = nullptr, *dp = nullptr, *Xcand = nullptr, *rhs_p = nullptr;
  double *Uraw = nullptr, *gc = nullptr, *b = nullptr, *Minv = nullptr, *rhs_c = nullptr;
  double *x = nullptr, *r = nullptr, *u = nullptr, *p = nullptr, *sv = nullptr,
         *wv = nullptr, *dots = nullptr, *part = nullptr;
  // camera-pass items (CamItems) of the current solve, and the point-range bounds of the
  // camera segments they are cut at
  int *item_off = nullptr, *rb = nullptr;
  int4* item_at = nullptr;
  int it_R = 1, it_cap = 0, it_nslot = 0, it_slots = 0, it_count = 0, it_K = 0;
  bool items_ok = false;   // the items match the current extraction (and it_R, it_K)

  // explicit reduced camera system (solver = BA_SOLVER_EXPLICIT), sized per extraction
  Arena ex;
  int64_t ex_cap = 0;                 // contributions the buffers hold
  int64_t ex_bytes = 0;               // bytes of the contribution-sized buffers
  int64_t ex_nc = 0, ex_nb = 0;       // contributions, off-diagonal blocks
  uint32_t *ex_key = nullptr, *ex_skey = nullptr;
  uint64_t *ex_val = nullptr, *ex_sval = nullptr;   // (a, b) point-major positions
  int* ex_pm_rank = nullptr;
  int64_t *ex_flag = nullptr, *ex_bidx = nullptr, *ex_cnt = nullptr, *ex_coff = nullptr;
  uint32_t* ex_bkey = nullptr;
  int64_t *ex_bstart = nullptr, *ex_row_ptr = nullptr;
  void* ex_sblk = nullptr;
  double* ex_scc = nullptr;
  void* ex_tmp = nullptr;
  size_t ex_tmp_bytes = 0;
  bool ex_valid = false;              // pattern of the current extraction

  // global positioning (allocated on its first step)
  double* gp_s = nullptr;                       // N scales, caller's observation order
  double* gp_scand = nullptr;                   // compact candidate scales
  void *gp_lin_pm = nullptr, *gp_lin_cm = nullptr, *gp_a_pm = nullptr, *gp_a_cm = nullptr;
  bool gp_ready = false;                        // scales initialised
  bool gp_lin_valid = false;                    // GP linearisation of the current estimate
  double gp_lam = 1e-3, gp_nu = 2.0, gp_last_decrease = 0.0;
  double *partials = nullptr, *scal = nullptr;
  double *grad_cams_d = nullptr, *grad_pts_d = nullptr;
  float *gxy_d = nullptr, *gdepth_d = nullptr;
  PcgState* pcg = nullptr;
  PcgState* pcg_diag = nullptr;   // state of the extra matvec that measures the true residual
  double* diag = nullptr;         // |b - S x|^2, |b|^2 of that product
  double* h_pin = nullptr;   // pinned host readback buffer
  hipEvent_t pcg_ev[2] = {nullptr, nullptr};   // the PCG state copies of two batches
  int pcg_pending = -1;   // batch whose state copy the LM step reads at its next sync
  hipEvent_t items_ev = nullptr;   // the item counts' copy after an item build
  bool items_pending = false;      // it_count / it_slots still the upper bounds

  // LM state
  double lam = 1e-3, nu = 2.0;
  bool lin_valid = false, ext_valid = false, step_valid = false, blocks_valid = false;
  int Ca = 0, Pa = 0, rounds = 0;
  int64_t Nh = 0, Nc = 0;
  double last_decrease = 0.0;   // per-observation actual reduction of the last step

  iba::DevLimits dl;   // compute units and LDS sizes of the context's device
  int device = 0;      // HIP device the context was created on
  void* scratch_dev = nullptr;   // that device's static scratch array (ba_lm_step_noalloc)
  // timing
  std::vector<KStat> stats;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;

  void release_explicit() {
    for (void* p : {(void*)ex_key, (void*)ex_val, (void*)ex_skey, (void*)ex_sval,
                    (void*)ex_flag, (void*)ex_bidx, (void*)ex_bkey, (void*)ex_bstart, ex_sblk,
                    ex_tmp})
      if (p) (void)hipFree(p);
    ex_key = ex_skey = ex_bkey = nullptr;
    ex_val = ex_sval = nullptr;
    ex_pm_rank = nullptr;
    ex_flag = ex_bidx = ex_cnt = ex_coff = ex_bstart = ex_row_ptr = nullptr;
    ex_sblk = ex_tmp = nullptr;
    ex_scc = nullptr;
    ex_tmp_bytes = 0;
    ex_cap = ex_nc = ex_nb = ex_bytes = 0;
    ex_valid = false;
    ex.release();
  }

  ~ba_ctx() {
    release_explicit();
    for (auto& pe : pending) {
      (void)hipEventDestroy(pe.a);
      (void)hipEventDestroy(pe.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
    if (items_ev) (void)hipEventDestroy(items_ev);
    for (auto e : pcg_ev)
      if (e) (void)hipEventDestroy(e);
    obs.release();
    par.release();
    if (h_pin) (void)hipHostFree(h_pin);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  size_t tsize() const { return opt.precision == BA_PRECISION_FP64 ? 8 : 4; }
  int need_pt() const { return opt.activity_rule == BA_ACTIVITY_LITERAL ? 1 : 3; }
  // camera unknowns: pose (6), plus the focal length when it is refined (7)
  int D = 6;
  int need_cam() const { return opt.activity_rule == BA_ACTIVITY_LITERAL ? 1 : D; }

  Model model() const {
    Model m;
    m.lam_d = have_priors ? lam_d : 0.0;
    m.huber = opt.huber_px;
    m.min_depth = opt.min_depth;
    m.filter_px = opt.filter_px;
    m.img_w = opt.img_w;
    m.img_h = opt.img_h;
    return m;
  }

  // ---------------------------------------------------------------- timing helpers
  int kid(const char* name) {
    for (size_t i = 0; i < stats.size(); ++i)
      if (stats[i].name == name) return int(i);
    stats.push_back(KStat{name});
    return int(stats.size() - 1);
  }
  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    return e;
  }
  // One kernel: its own start and end timestamps (events handed to the launch itself).
  template <class F>
  void timed(const char* name, double bytes, int pcg_iter, F&& launch) {
    if (!opt.timing) {
      launch();
      HIP_LAUNCH_CHECK();
      return;
    }
    Pending pe{kid(name), get_event(), get_event(), bytes, pcg_iter};
    const int64_t before = iba::launches_issued();
    iba::set_launch_events(pe.a, pe.b);
    launch();
    iba::set_launch_events(nullptr, nullptr);
    HIP_LAUNCH_CHECK();
    const int64_t n = iba::launches_issued() - before;
    if (n == 0) {   // nothing to do for an empty range
      pool.push_back(pe.a);
      pool.push_back(pe.b);
      return;
    }
    if (n != 1) throw BaError{BA_ERR_STATE, std::string("internal: timed scope ") + name +
                                                " launched several kernels"};
    pending.push_back(pe);
  }
  // Several kernels: events recorded in the stream around them.
  template <class F>
  void timed_multi(const char* name, double bytes, F&& launch) {
    if (!opt.timing) {
      launch();
      HIP_LAUNCH_CHECK();
      return;
    }
    Pending pe{kid(name), get_event(), get_event(), bytes, -1};
    HIP_CHECK(hipEventRecord(pe.a, stream));
    launch();
    HIP_LAUNCH_CHECK();
    HIP_CHECK(hipEventRecord(pe.b, stream));
    pending.push_back(pe);
  }
  // After a stream sync: fold event pairs into the statistics. PCG launches beyond the
  // iteration that converged only test the done flag and are not counted.
  void flush_timing(int pcg_iters_done) {
    for (auto& pe : pending) {
      if (pe.pcg_iter < 0 || pe.pcg_iter < pcg_iters_done) {
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, pe.a, pe.b));
        KStat& s = stats[pe.kid];
        s.launches += 1;
        s.ms += ms;
        s.bytes += pe.bytes;
      }
      pool.push_back(pe.a);
      pool.push_back(pe.b);
    }
    pending.clear();
  }

  void sync() { HIP_CHECK(hipStreamSynchronize(stream)); }
  void to_device(void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return;
    HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, stream));
  }
};

namespace {

// Copy caller memory (host or device) into a host vector.
template <typename T>
void fetch(ba_ctx& c, std::vector<T>& dst, const T* src, size_t n) {
  dst.resize(n);
  if (n == 0) return;
  HIP_CHECK(hipMemcpyAsync(dst.data(), src, n * sizeof(T), hipMemcpyDefault, c.stream));
  c.sync();
}

template <typename T>
void store(ba_ctx& c, T* dst, const T* src_host, size_t n) {
  if (n == 0) return;
  HIP_CHECK(hipMemcpyAsync(dst, src_host, n * sizeof(T), hipMemcpyDefault, c.stream));
  c.sync();
}

template <typename T>
void download(ba_ctx& c, std::vector<T>& dst, const T* dev, size_t n) {
  dst.resize(n);
  if (n == 0) return;
  HIP_CHECK(hipMemcpyAsync(dst.data(), dev, n * sizeof(T), hipMemcpyDeviceToHost, c.stream));
  c.sync();
}

ba_status fail(ba_ctx* c, ba_status code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

template <class F>
ba_status guarded(ba_ctx* c, F&& f) {
  if (!c) return BA_ERR_ARG;
  try {
    return f();
  } catch (const BaError& e) {
    c->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return BA_ERR_OOM;
  } catch (const std::exception& e) {
    c->err = e.what();
    return BA_ERR_DEVICE;
  }
}

// ------------------------------------------------------------------ buffers
// Most camera-pass items a solve can have (CamItems: R Ca + nchunks, R <= 8).
size_t item_slots(int C) { return size_t(kMaxRanges) * size_t(C) + kCamChunks; }
// Partial values per item slot: the camera assembly's 2 (D (D + 1) / 2 + D) (item-major), or
// the PCG camera pass's D + 1 rows (which also covers global positioning, D = 3).
size_t part_rows(int D) {
  return std::max(2 * (size_t(D) * (D + 1) / 2 + D), size_t(D) + 1);
}

void alloc_obs_buffers(ba_ctx& c) {
  c.release_explicit();
  c.obs.release();
  Arena& A = c.obs;
  const int64_t N = c.N;
  const int C = c.C, P = c.P;
  const size_t ts = c.tsize();
  c.pm_cam = A.alloc<int>(N);
  c.pm_pt = A.alloc<int>(N);
  c.pm_orig = A.alloc<int>(N);
  c.pm_xy = A.alloc<float2>(N);
  c.pm_depth = A.alloc<float>(N);
  c.pt_off = A.alloc<int>(P + 1);
  c.cm_off = A.alloc<int>(C + 1);
  c.inv_cm = A.alloc<int>(N);
  c.cm_cam = A.alloc<int>(N);
  c.pt_user_d = A.alloc<int>(P);
  c.vrow = A.alloc<uint8_t>(N);
  c.vrow_cm = A.alloc<uint8_t>(N);
  c.act_c = A.alloc<uint8_t>(C);
  c.act_p = A.alloc<uint8_t>(P);
  c.rank_c = A.alloc<int>(C + 1);
  c.rank_p = A.alloc<int>(P + 1);
  c.pos_pm = A.alloc<int>(N + 1);
  c.pos_cm = A.alloc<int>(N + 1);
  if (std::max<int64_t>({N, int64_t(P), int64_t(C)}) + 1 > int64_t(INT32_MAX))
    throw BaError{BA_ERR_ARG, "more than 2^31 - 2 observations, points or cameras"};
  c.scan_temp_size = scan_temp_bytes(std::max<int64_t>({N, int64_t(P), int64_t(C)}));
  c.scan_temp = A.alloc<char>(c.scan_temp_size);
  c.flags = A.alloc<int>(4);
  c.cam_hat = A.alloc<int>(N);
  c.orig_hat = A.alloc<int>(N);
  c.xy_hat = A.alloc<float2>(N);
  c.depth_hat = A.alloc<float>(N);
  c.off_hat = A.alloc<int>(P + 1);
  c.pt_src = A.alloc<int>(P);
  c.cam_src = A.alloc<int>(C);
  c.slot_all = A.alloc<int>(C);
  c.camd_hat = A.alloc<Cam<double>>(C);
  c.camf_hat = A.alloc<Cam<float>>(C);
  c.cm_off_hat = A.alloc<int>(C + 1);
  c.cm_pt = A.alloc<int>(N);
  c.pm_cm = A.alloc<int>(N);
  c.Xd = A.alloc<double>(3 * size_t(P));
  c.Xf = A.alloc<float>(3 * size_t(P));
  c.w = A.alloc<char>(ts * N);
  c.xcw = A.alloc<char>(4 * ts * N);
  c.cm_e = A.alloc<char>(4 * ts * N);
  // the point-major Jacobian stream: read by the float64 point pass and by the explicit
  // system's block assembly (the float32 point pass forms X_c itself)
  c.pm_xcw = (ts == 8 || c.opt.solver == BA_SOLVER_EXPLICIT) ? A.alloc<char>(4 * ts * N)
                                                             : nullptr;
  c.eh = nullptr;
  c.cm_eh = nullptr;
  c.ce = nullptr;
  c.cm_ce = nullptr;
  c.gp_s = nullptr;
  c.gp_ready = false;
  c.V = A.alloc<char>(sizeof(double) * 6 * P);
  c.Vinv = A.alloc<char>(ts * 6 * P);
  c.prec = A.alloc<char>((ts == 8 ? sizeof(PtRec<double>) : sizeof(PtRec<float>)) * P);
  c.zq = A.alloc<char>(3 * ts * std::max<int64_t>(N, P));   // per point, or per position (GP)
  const size_t ns = size_t(c.D) * (c.D + 1) / 2;   // entries of a symmetric camera block
  const size_t nd = size_t(c.D);
  c.Ustar = A.alloc<char>(ts * ns * C);
  c.mvt = A.alloc<char>(ts * 20 * C);   // MvCam or MvCamF records (at most 20 T each)
  c.gp = A.alloc<double>(3 * size_t(P));
  c.hp = A.alloc<double>(3 * size_t(P));
  c.dp = A.alloc<double>(3 * size_t(P));
  c.Xcand = A.alloc<double>(3 * size_t(P));
  c.rhs_p = A.alloc<double>(3 * size_t(P));
  c.Uraw = A.alloc<double>(ns * size_t(C));
  c.gc = A.alloc<double>(nd * size_t(C));
  c.b = A.alloc<double>(nd * size_t(C));
  c.Minv = A.alloc<double>(ns * size_t(C));
  c.rhs_c = A.alloc<double>(nd * size_t(C));
  c.x = A.alloc<double>(nd * size_t(C));
  c.r = A.alloc<double>(nd * size_t(C));
  c.u = A.alloc<double>(nd * size_t(C));
  c.p = A.alloc<double>(nd * size_t(C));
  c.sv = A.alloc<double>(nd * size_t(C));
  c.wv = A.alloc<double>(nd * size_t(C));          // U* u of the current PCG direction
  c.dots = A.alloc<double>(2 * 3 * size_t(C));     // per-camera terms, two parities
  c.part = A.alloc<double>(part_rows(c.D) * item_slots(C));   // item partials
  c.items_ok = false;
  c.item_off = A.alloc<int>(size_t(C) + 2);
  c.item_at = A.alloc<int4>(size_t(kMaxRanges) * (size_t(C) + kCamChunks));
  c.rb = A.alloc<int>(size_t(kMaxRanges) * C);
  // 5 sums per workgroup; the global-positioning candidate runs up to 16 lanes per point
  c.partials = A.alloc<double>(5 * (size_t(P) * 16 / kBlock + 16));
  c.scal = A.alloc<double>(16);
  c.pcg = A.alloc<PcgState>(1);
  c.pcg_diag = A.alloc<PcgState>(1);
  c.diag = A.alloc<double>(4);
  c.grad_cams_d = nullptr;
  c.grad_pts_d = nullptr;
  c.gxy_d = nullptr;
  c.gdepth_d = nullptr;
}

void ensure_adjoint_buffers(ba_ctx& c) {
  if (c.eh) return;
  const size_t ts = c.tsize();
  c.eh = c.obs.alloc<char>(ts * 3 * size_t(c.N));
  c.cm_eh = c.obs.alloc<char>(ts * 3 * size_t(c.N));
  c.ce = c.obs.alloc<char>(ts * 3 * size_t(c.N));
  c.cm_ce = c.obs.alloc<char>(ts * 3 * size_t(c.N));
  c.grad_cams_d = c.obs.alloc<double>(7 * size_t(c.C));
  c.grad_pts_d = c.obs.alloc<double>(3 * size_t(c.P));
  c.gxy_d = c.obs.alloc<float>(2 * size_t(c.N));
  c.gdepth_d = c.obs.alloc<float>(size_t(c.N));
}

template <typename T>
Compact<T> compact_view(ba_ctx& c) {
  Compact<T> cp;
  cp.Pa = c.Pa;
  cp.Ca = c.Ca;
  cp.Cf = c.n_fixed;
  cp.off = c.off_hat;
  cp.cam = c.cam_hat;
  cp.xy = c.xy_hat;
  cp.depth = c.depth_hat;
  cp.cam_src = c.cam_src;
  cp.cm_off = c.cm_off_hat;
  cp.cm_pt = c.cm_pt;
  cp.pm_cm = c.pm_cm;
  cp.Xd = c.Xd;
  cp.camd = c.camd_hat;
  if constexpr (sizeof(T) == 8) {
    cp.Xt = reinterpret_cast<const T*>(c.Xd);
    cp.camt = reinterpret_cast<const Cam<T>*>(c.camd_hat);
  } else {
    cp.Xt = reinterpret_cast<const T*>(c.Xf);
    cp.camt = reinterpret_cast<const Cam<T>*>(c.camf_hat);
  }
  return cp;
}

template <typename T>
ObsMetric<T> metric_view(ba_ctx& c) {
  ObsMetric<T> om;
  om.w = static_cast<T*>(c.w);
  om.xcw = static_cast<V4<T>*>(c.xcw);
  om.cm_e = static_cast<V4<T>*>(c.cm_e);
  om.pm_xcw = static_cast<V4<T>*>(c.pm_xcw);
  om.eh = static_cast<T*>(c.eh);
  om.cm_eh = static_cast<T*>(c.cm_eh);
  om.ce = c.ce_on ? static_cast<T*>(c.ce) : nullptr;
  om.cm_ce = c.ce_on ? static_cast<T*>(c.cm_ce) : nullptr;
  return om;
}

// The camera-pass items of the current solve.
CamItems items_view(const ba_ctx& c) {
  CamItems it;
  it.R = c.it_R;
  it.cap = c.it_cap;
  it.off = c.item_off;
  it.at = c.item_at;
  it.slots = c.it_slots;
  return it;
}

// Sets up the items of a solve over R point ranges (8 for the matrix-free LM passes: the
// eighths of the point ranks the point pass gives the XCDs, ppx = ceil(Pa / 8) each; 1 for
// whole camera segments) and returns the partial-slot count; the PCG init builds them.
int plan_items(ba_ctx& c, int R, int nch) {
  c.it_R = R;
  c.it_cap = c.Ca + nch;
  c.it_nslot = R * c.Ca + nch;
  c.it_slots = c.it_cap;
  if (R > 1)
    launch_range_bounds(c.stream, c.Ca, R, (c.Pa + R - 1) / R, c.cm_off_hat, c.cm_pt, c.rb);
  return c.it_nslot;
}

// After the item build: the item count and the largest item count of a range, which size the
// update's reduction and the camera-pass grids. They are copied with an event and read when
// the PCG starts (resolve_items), by which time the stream is busy with the work queued since
// the build; until then it_count and it_slots hold their upper bounds (the camera assembly's
// grids cover cap slots per range, the slots past a range's last item return at once).
void request_item_counts(ba_ctx& c) {
  HIP_CHECK(hipMemcpyAsync(c.h_pin + 24, c.item_off + c.Ca, 2 * sizeof(int),
                           hipMemcpyDeviceToHost, c.stream));
  HIP_CHECK(hipEventRecord(c.items_ev, c.stream));
  c.it_count = c.it_nslot;
  c.it_slots = c.it_cap;
  c.items_pending = true;
}

void resolve_items(ba_ctx& c) {
  if (!c.items_pending) return;
  HIP_CHECK(hipEventSynchronize(c.items_ev));
  int n[2] = {0, 0};
  std::memcpy(n, c.h_pin + 24, sizeof(n));
  c.it_count = std::max(0, std::min(n[0], c.it_nslot));
  c.it_slots = std::max(0, std::min(n[1], c.it_cap));
  c.items_pending = false;
}

// Builds the camera-pass items (R ranges, at most K positions each, nch = ceil(Nc / K)) unless
// the current ones are those; returns the partial-slot count.
int ensure_items(ba_ctx& c, int R, int K, int nch) {
  if (c.items_ok && c.it_R == R && c.it_K == K) return c.it_nslot;
  plan_items(c, R, nch);
  launch_build_items(c.stream, c.Ca, c.cm_off_hat, c.rb, K, items_view(c));
  HIP_LAUNCH_CHECK();
  request_item_counts(c);
  if (c.opt.timing) resolve_items(c);   // exact byte models; timing syncs anyway
  c.it_K = K;
  c.items_ok = true;
  return c.it_nslot;
}

// ------------------------------------------------------------------ extraction
// Validity, activity fixpoint, ranks and compaction at the current parameters.
// Dynamic parameter extraction. gp selects the global-positioning rules: validity is finite
// data only, 3 rows per pinned and 2 per free observation, cameras need 3 rows.
void extract(ba_ctx& c, bool gp = false) {
  c.gp_lin_valid = false;   // the compaction buffers are rebuilt
  c.items_ok = false;
  const Model m = c.model();
  hipStream_t s = c.stream;
  const int64_t N = c.N;
  c.timed("cam_table", double(c.C) * (56 + 24 + 120 + 60), -1,
          [&] { launch_cam_table(s, c.C, c.d_cams, c.d_intr, c.d_camd, c.d_camf); });
  if (gp)
    c.timed("gp_validate", double(N) * (8 + 4 + 4 + 1 + 1), -1, [&] {
      launch_gp_validate(s, N, c.pm_xy, c.pm_depth, c.inv_cm, c.vrow, c.vrow_cm);
    });
  else
    c.timed("validate", double(N) * (4 + 4 + 8 + 4 + 24 + 1 + 4 + 1), -1, [&] {
      launch_validate_lds(s, N, c.C, m, c.pm_cam, c.pm_pt, c.pm_xy, c.pm_depth, c.d_pts,
                          c.d_camd, c.inv_cm, c.vrow, c.vrow_cm, c.dl, 1);
    });
  const int need_cam = gp ? 3 : c.need_cam();
  const int need_pt = gp ? 3 : c.need_pt();
  // two rounds per host check: a round at the fixpoint changes nothing, so the second round
  // of a pair is harmless when the first one settled it (flags[0] and flags[2] say whether
  // each round changed anything)
  int rounds = 0;
  while (true) {
    for (int k = 0; k < 2; ++k) {
      int* changed = c.flags + 2 * k;
      HIP_CHECK(hipMemsetAsync(changed, 0, sizeof(int), s));
      c.timed("cam_rows", double(N) * 1, -1, [&] {
        launch_cam_rows(s, c.C, c.cm_off, c.vrow_cm, c.d_fixed, need_cam, c.act_c);
      });
      c.timed("point_rows_prune", double(N) * 5 + double(c.P) * 5, -1, [&] {
        launch_point_rows_prune(s, c.P, c.pt_off, c.pm_cam, c.act_c, c.d_fixed, need_pt,
                                c.inv_cm, c.vrow, c.vrow_cm, c.act_p, changed);
      });
    }
    HIP_CHECK(hipMemcpyAsync(c.h_pin, c.flags, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    c.sync();
    int f[3] = {0, 0, 0};
    std::memcpy(f, c.h_pin, sizeof(f));
    if (!f[0]) {
      rounds += 1;
      break;
    }
    rounds += 2;
    if (!f[2]) break;
    if (rounds > 1000000) throw BaError{BA_ERR_DEVICE, "activity fixpoint did not settle"};
  }
  c.rounds = rounds;
  c.timed_multi("scan", double(c.C) * 5 + double(c.P) * 5 + double(N) * 14, [&] {
    const size_t tb = c.scan_temp_size;
    HIP_CHECK(launch_scan_u8(s, c.C, c.act_c, c.rank_c, c.scan_temp, tb));
    HIP_CHECK(launch_scan_u8(s, c.P, c.act_p, c.rank_p, c.scan_temp, tb));
    HIP_CHECK(launch_scan_u8(s, N, c.vrow, c.pos_pm, c.scan_temp, tb));
    HIP_CHECK(launch_scan_cm(s, N, c.vrow_cm, c.cm_cam, c.d_fixed, c.pos_cm, c.scan_temp, tb));
  });
  int* hp = reinterpret_cast<int*>(c.h_pin);
  HIP_CHECK(hipMemcpyAsync(hp + 0, c.rank_c + c.C, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(hp + 1, c.rank_p + c.P, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(hp + 2, c.pos_pm + N, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(hp + 3, c.pos_cm + N, sizeof(int), hipMemcpyDeviceToHost, s));
  c.sync();
  c.Ca = hp[0];
  c.Pa = hp[1];
  c.Nh = hp[2];
  c.Nc = hp[3];
  c.timed_multi("compact", double(N) * 72 + double(c.P) * 60, [&] {
    launch_compact_cams(s, c.C, c.act_c, c.rank_c, c.d_fixed, c.d_fixed_rank, c.cm_off,
                        c.pos_cm, c.slot_all, c.cam_src, c.cm_off_hat);
    launch_compact_cam_table(s, c.Ca + c.n_fixed, c.cam_src, c.d_camd, c.d_camf, c.camd_hat,
                             c.camf_hat);
    launch_compact_points(s, c.P, c.act_p, c.rank_p, c.pt_off, c.pos_pm, c.d_pts, c.pt_src,
                          c.off_hat, c.Xd, c.Xf);
    launch_compact_obs(s, N, c.vrow, c.pos_pm, c.pm_cam, c.slot_all, c.pm_xy, c.pm_depth,
                       c.pm_orig, c.Ca, c.inv_cm, c.pos_cm, c.pm_pt, c.rank_p, c.cam_hat,
                       c.xy_hat, c.depth_hat, c.orig_hat, c.pm_cm, c.cm_pt);
    if (gp)
      ;   // the global-positioning matvec records hold u only, set by the PCG init
    else if (c.tsize() == 8)
      launch_mv_table<double>(s, c.D, c.Ca + c.n_fixed, c.camd_hat, c.mvt);
    else
      launch_mv_table<float>(s, c.D, c.Ca + c.n_fixed, c.camd_hat, c.mvt);
  });
  c.ext_valid = true;
}

// Algorithmic bytes of the two PCG passes (unique data each must touch once).
// Point pass: per observation its slot and, in float32, its weight (X_c is formed from the
// point) or, in float64, its (X_c, w) 4-vector; per point the CSR offset, Vinv, in float32 the
// point, and its z 3-vector written; every matvec record once.
double bytes_schur_point(const ba_ctx& c) {
  const double ts = double(c.tsize());
  const bool form = ts == 4;
  const double rec = form || c.D == 7 ? 20 : 16;   // matvec record values
  return double(c.Nh) * (4 + (form ? 1 : 4) * ts) +
         double(c.Pa) * (4 + (form ? 9 : 6) * ts + 3 * ts) + double(c.Ca) * rec * ts;
}
// Camera pass: per camera-major position the (X_c, w) 4-vector and the point rank; the z
// vectors once (each XCD reads its eighth of the points, gathered through its L2); per item
// its bounds, camera, table entry and u, and its D + 1 partial values written.
double bytes_schur_cam(const ba_ctx& c) {
  const double ts = double(c.tsize());
  const double D = c.D;
  int K = 0, nch = 0;
  cam_chunking(c.Nc, K, nch);
  const double items = double(kMaxRanges) * c.Ca + nch;
  return double(c.Nc) * (4 * ts + 4) + double(c.Pa) * 3 * ts +
         items * (16 + 15 * ts + D * 8 + (D + 1) * 8);
}
// PCG update: per camera its terms (read and written), offsets, M^-1, U*, the vectors
// p s x r u and U* u (read and written) and its matvec record's u; every partial slot once.
double bytes_pcg_update(const ba_ctx& c) {
  const double ts = double(c.tsize());
  const double D = c.D, ns = D * (D + 1) / 2;
  int K = 0, nch = 0;
  cam_chunking(c.Nc, K, nch);
  return double(c.Ca) * (2 * 3 * 8 + 4 + ns * 8 + ns * ts + 2 * 6 * D * 8 + D * ts) +
         (double(kMaxRanges) * c.Ca + nch) * (D + 1) * 8;
}
// Smallest LM damping. In mixed precision the damped blocks U*, V*^-1 and the matvec are
// float32: a Marquardt damping of the order of their rounding (6e-8) amplified by the
// summation over a camera's observations is lost, the damped reduced system is then singular
// or indefinite at float32 resolution along its weakest directions (the gauge, the depth of
// far points), and its PCG diverges into non-positive curvature. Mixed precision therefore
// keeps the damping at 1e-5 or more; float64 uses lambda_min as given.
constexpr double kMixedLambdaFloor = 1e-5;
double lambda_floor(const ba_ctx& c) {
  return c.opt.precision == BA_PRECISION_MIXED ? std::max(c.opt.lambda_min, kMixedLambdaFloor)
                                               : c.opt.lambda_min;
}

int lanes_per_point(const ba_ctx& c) {
  const double mean = c.Pa > 0 ? double(c.Nh) / c.Pa : 1.0;
  return mean <= 2.5 ? 2 : mean <= 4.5 ? 4 : mean <= 9.0 ? 8 : 16;
}

template <typename T>
void linearize(ba_ctx& c, bool adj) {
  c.gp_lin_valid = false;   // shares the point-gradient and scalar buffers
  hipStream_t s = c.stream;
  const Model m = c.model();
  Compact<T> cp = compact_view<T>(c);
  ObsMetric<T> om = metric_view<T>(c);
  const double ts = double(sizeof(T));
  // per observation: slot, xy, depth and camera-major position read; w written (and the
  // point-major (X_c, w) where kept), plus the camera-major (X_c, w) and e (and eh) for solve
  // cameras
  const double pm_stream = c.pm_xcw ? 4 * ts : 0.0;
  int nb = 0;
  c.timed("lin_point", double(c.Nh) * (4 + 8 + 4 + 4 + ts + pm_stream + (adj ? 3 * ts : 0)) +
                           double(c.Nc) * (8 * ts + (adj ? 3 * ts : 0)) +
                           double(c.Pa) * (4 + 24 + 48 + 24) + double(c.C) * 120,
          -1, [&] {
            nb = launch_lin_point<T>(s, adj, lanes_per_point(c), m, cp, om,
                                     static_cast<double*>(c.V), c.gp, c.partials, c.dl);
          });
  launch_reduce_partials(s, nb, 3, c.partials, 0x4u, 0, nullptr, nullptr, c.scal);
  HIP_LAUNCH_CHECK();
}

bool explicit_solver(const ba_ctx& c) { return c.opt.solver == BA_SOLVER_EXPLICIT; }

// Block pattern of the reduced camera system for the current extraction: every ordered pair of
// distinct solve-camera observations of a point is one contribution, keyed by its camera pair;
// a stable sort groups the contributions of each block in point order.
template <typename T>
void build_schur_pattern(ba_ctx& c) {
  hipStream_t s = c.stream;
  Compact<T> cp = compact_view<T>(c);
  const int Pa = c.Pa;
  if (!c.ex_pm_rank) {
    c.ex_pm_rank = c.ex.alloc<int>(size_t(c.N));
    c.ex_cnt = c.ex.alloc<int64_t>(size_t(c.P) + 1);
    c.ex_coff = c.ex.alloc<int64_t>(size_t(c.P) + 1);
    c.ex_row_ptr = c.ex.alloc<int64_t>(size_t(c.C) + 1);
    c.ex_scc = c.ex.alloc<double>(size_t(c.D) * (c.D + 1) / 2 * size_t(c.C));
  }
  HIP_CHECK(hipMemsetAsync(c.ex_cnt + Pa, 0, sizeof(int64_t), s));
  c.timed_multi("schur_pattern", double(c.Nh) * 8 + double(Pa) * 16, [&] {
    launch_pair_counts<T>(s, cp, c.ex_cnt, c.ex_pm_rank);
  });
  size_t tb = exclusive_sum_temp_bytes(Pa + 1);
  void* tmp = nullptr;
  Arena scan_tmp;
  tmp = scan_tmp.alloc<char>(tb);
  HIP_CHECK(exclusive_sum(tmp, tb, c.ex_cnt, c.ex_coff, Pa + 1, s));
  int64_t nc = 0;
  HIP_CHECK(hipMemcpyAsync(&nc, c.ex_coff + Pa, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  c.sync();
  scan_tmp.release();
  if (nc >= (int64_t(1) << 31))
    throw BaError{BA_ERR_ARG, "explicit reduced system: more than 2^31 block contributions"};
  if (int64_t(c.Ca) * int64_t(c.Ca) >= (int64_t(1) << 32))
    throw BaError{BA_ERR_ARG, "explicit reduced system: too many cameras for 32-bit block keys"};
  c.ex_nc = nc;
  c.ex_nb = 0;
  int end_bit = 1;
  while ((uint64_t(1) << end_bit) < uint64_t(c.Ca) * uint64_t(c.Ca)) ++end_bit;
  if (nc > c.ex_cap) {
    // contribution-sized buffers grow with the pattern (25 % headroom)
    const int64_t cap = nc + nc / 4 + 1024;
    for (void* p : {(void*)c.ex_key, (void*)c.ex_val, (void*)c.ex_skey, (void*)c.ex_sval,
                    (void*)c.ex_flag, (void*)c.ex_bidx, (void*)c.ex_bkey, (void*)c.ex_bstart,
                    c.ex_sblk, c.ex_tmp})
      if (p) (void)hipFree(p);
    c.ex_bytes = 0;
    auto grab = [&](size_t bytes) {
      void* p = nullptr;
      bytes = std::max<size_t>(bytes, 256);
      if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw BaError{BA_ERR_OOM, "explicit reduced system: device allocation failed"};
      }
      c.ex_bytes += int64_t(bytes);
      return p;
    };
    c.ex_key = static_cast<uint32_t*>(grab(4 * size_t(cap)));
    c.ex_val = static_cast<uint64_t*>(grab(8 * size_t(cap)));
    c.ex_skey = static_cast<uint32_t*>(grab(4 * size_t(cap)));
    c.ex_sval = static_cast<uint64_t*>(grab(8 * size_t(cap)));
    c.ex_flag = static_cast<int64_t*>(grab(8 * size_t(cap)));
    c.ex_bidx = static_cast<int64_t*>(grab(8 * size_t(cap)));
    c.ex_bkey = static_cast<uint32_t*>(grab(4 * size_t(cap)));
    c.ex_bstart = static_cast<int64_t*>(grab(8 * (size_t(cap) + 1)));
    c.ex_sblk = grab(size_t(c.tsize()) * size_t(c.D) * c.D * size_t(cap));
    c.ex_tmp_bytes = std::max(sort_pairs64_temp_bytes(int(cap), 32),
                              exclusive_sum_temp_bytes(int(cap)));
    c.ex_tmp = grab(c.ex_tmp_bytes);
    c.ex_cap = cap;
  }
  if (nc > 0) {
    c.timed_multi("schur_pattern", double(Pa) * 24 + double(nc) * 12, [&] {
      launch_pair_keys<T>(s, cp, c.ex_coff, c.ex_key, c.ex_val);
    });
    c.timed_multi("schur_pattern", double(nc) * 48, [&] {
      HIP_CHECK(sort_pairs64(c.ex_tmp, c.ex_tmp_bytes, c.ex_key, c.ex_skey, c.ex_val,
                             c.ex_sval, int(nc), end_bit, s));
    });
    launch_run_flags(s, nc, c.ex_skey, c.ex_flag);
    HIP_CHECK(exclusive_sum(c.ex_tmp, c.ex_tmp_bytes, c.ex_flag, c.ex_bidx, int(nc), s));
    int64_t tail[2] = {0, 0};
    HIP_CHECK(hipMemcpyAsync(&tail[0], c.ex_bidx + nc - 1, sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(&tail[1], c.ex_flag + nc - 1, sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
    c.sync();
    c.ex_nb = tail[0] + tail[1];
    launch_block_list(s, nc, c.ex_skey, c.ex_flag, c.ex_bidx, c.ex_bkey, c.ex_bstart);
    HIP_CHECK(hipMemcpyAsync(c.ex_bstart + c.ex_nb, &nc, sizeof(int64_t), hipMemcpyHostToDevice,
                             s));
  }
  launch_block_rows(s, c.Ca, c.ex_nb, c.ex_bkey, c.ex_row_ptr);
  HIP_LAUNCH_CHECK();
  c.sync();   // the host values above are stack copies
  c.ex_valid = true;
}

// Off-diagonal blocks at the current damping (V*^-1 from the point setup).
template <typename T>
void assemble_schur_blocks(ba_ctx& c) {
  if (c.ex_nb == 0) return;
  const double ts = double(c.tsize());
  const double DD = double(c.D) * c.D;
  c.timed("schur_blocks",
          double(c.ex_nc) * (8 + 4 + 2 * 4 * ts + 6 * ts) + double(c.ex_nb) * (4 + 8 + DD * ts),
          -1, [&] {
            launch_schur_blocks<T>(c.stream, c.D, c.model(), compact_view<T>(c), metric_view<T>(c),
                                   static_cast<const T*>(c.Vinv), c.ex_pm_rank, c.ex_nb,
                                   c.ex_bkey, c.ex_bstart, c.ex_sval,
                                   static_cast<T*>(c.ex_sblk));
          });
}

// Damping-dependent setup: point inverses, camera blocks, Schur RHS, preconditioner.
template <typename T>
void setup_system(ba_ctx& c, bool adj, double lam, const double* rhs_c, const double* rhs_p) {
  hipStream_t s = c.stream;
  const Model m = c.model();
  Compact<T> cp = compact_view<T>(c);
  ObsMetric<T> om = metric_view<T>(c);
  const double ts = double(sizeof(T));
  HIP_CHECK(hipMemsetAsync(c.flags + 1, 0, sizeof(int), s));
  c.timed("point_damp", double(c.Pa) * (48 + 24 + 6 * ts + 24 + double(sizeof(PtRec<T>))), -1,
          [&] {
    launch_point_damp<T>(s, c.Pa, lam, c.opt.diag_min, c.opt.diag_max,
                         static_cast<const double*>(c.V), c.gp, rhs_p, static_cast<T*>(c.Vinv),
                         c.hp, static_cast<PtRec<T>*>(c.prec), c.flags + 1);
  });
  if (c.Ca == 0) return;
  // the camera-pass items of this extraction (the PCG reuses them)
  int K = 0, nch = 0;
  cam_chunking(c.Nc, K, nch);
  const int nslot = ensure_items(c, kMaxRanges, K, nch);
  const CamItems items = items_view(c);
  const double ns = double(c.D) * (c.D + 1) / 2, rows = 2 * (ns + c.D);
  // per camera-major position the point rank and the (X_c, w) stream (+ eh); every point
  // record once; per item its record and its rows
  c.timed("cam_schur_items",
          double(c.Nc) * (4 + 4 * ts + (adj ? 3 * ts : 0)) +
              double(c.Pa) * double(sizeof(PtRec<T>)) + double(c.it_count) * (16 + 4 * rows),
          -1, [&] {
            launch_cam_items<T>(s, adj, true, c.D, m, cp, om,
                                static_cast<const PtRec<T>*>(c.prec), items, nslot, c.part,
                                c.dl);
          });
  // per camera-major position the (X_c, w) and e streams (+ eh); per item its record and rows
  c.timed("cam_u_items",
          double(c.Nc) * (8 * ts + (adj ? 3 * ts : 0)) + double(c.it_count) * (16 + 4 * rows), -1,
          [&] {
            launch_cam_items<T>(s, adj, false, c.D, m, cp, om, nullptr, items, nslot, c.part,
                                c.dl);
          });
  // the item rows; per camera its blocks written
  c.timed("cam_assemble",
          double(c.it_count) * 8 * rows + double(c.Ca) * (ns * (16 + ts) + c.D * 8 * 2 + 8), -1,
          [&] {
            launch_cam_assemble<T>(s, c.D, c.Ca, lam, c.opt.diag_min, c.opt.diag_max,
                                   c.item_off, c.part, rhs_c, c.Uraw,
                                   static_cast<T*>(c.Ustar), c.gc, c.b, c.Minv,
                                   explicit_solver(c) && !adj ? c.ex_scc : nullptr);
          });
}

// Runs PCG iterations in batches of pcg_check_every, batch(it0, it1) enqueuing iterations
// [it0, it1). The host reads the device-side state after each batch while the next batch is
// already queued (two pinned slots, one event each), so the GPU does not wait for the check;
// iterations enqueued after convergence return at their first instruction. Returns the state
// after the last batch that did work; with defer, once every iteration is queued it returns
// without waiting for them and leaves the last state's copy to the caller's next stream sync
// (c.pcg_pending names its slot, pcg_slot).
static_assert(sizeof(PcgState) <= 16 * sizeof(double), "a pinned slot holds one state");
double* pcg_slot(ba_ctx& c, int k) { return c.h_pin + 32 + 16 * (k & 1); }

template <class Batch>
PcgState pcg_batches(ba_ctx& c, int max_iters, Batch&& batch, bool defer = false) {
  const int every = std::max(1, c.opt.pcg_check_every);
  hipStream_t s = c.stream;
  int it = 0, n = 0;   // iterations and batches enqueued
  auto slot = [&](int k) { return pcg_slot(c, k); };
  auto enqueue = [&] {
    const int it1 = std::min(max_iters, it + every);
    batch(it, it1);
    it = it1;
    HIP_CHECK(hipMemcpyAsync(slot(n), c.pcg, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipEventRecord(c.pcg_ev[n & 1], s));
    ++n;
  };
  PcgState st{};
  auto read = [&](int k) {
    HIP_CHECK(hipEventSynchronize(c.pcg_ev[k & 1]));
    std::memcpy(&st, slot(k), sizeof(PcgState));
  };
  enqueue();
  while (true) {
    if (it >= max_iters) {   // every iteration is queued: the last batch's state
      if (defer)
        c.pcg_pending = n - 1;
      else
        read(n - 1);
      break;
    }
    enqueue();
    read(n - 2);
    if (st.done) break;   // the batch just queued returns at once
  }
  return st;
}

// PCG on the camera Schur complement; returns the iteration count (pcg_batches).
template <typename T>
int run_pcg(ba_ctx& c, bool adj, double rel_tol, int max_iters, PcgState* out_state,
            bool defer = false) {
  hipStream_t s = c.stream;
  const Model m = c.model();
  Compact<T> cp = compact_view<T>(c);
  ObsMetric<T> om = metric_view<T>(c);
  PcgState st{};
  if (c.Ca == 0) {
    *out_state = st;
    out_state->done = 1;
    return 0;
  }
  void* mvt = c.mvt;
  const T* Ustar = static_cast<const T*>(c.Ustar);
  int K = 0, nch = 0;
  cam_chunking(c.Nc, K, nch);
  const bool expl = explicit_solver(c) && !adj;
  if (expl) {   // one item per camera: the product of the explicit system is its partial
    K = std::numeric_limits<int>::max() / 2;
    nch = 0;
  }
  const int nslot = ensure_items(c, expl ? 1 : kMaxRanges, K, nch);
  resolve_items(c);
  launch_pcg_init<T>(s, c.D, c.Ca, c.b, c.Minv, Ustar, c.x, c.r, c.u, c.p, c.sv, c.wv, c.dots,
                     mvt, c.pcg, rel_tol * rel_tol, max_iters);
  HIP_LAUNCH_CHECK();
  const CamItems items = items_view(c);
  const double bp = bytes_schur_point(c), bc = bytes_schur_cam(c), bu = bytes_pcg_update(c);
  // explicit product: every block (D x D values and its key) and the row pointers once, the
  // camera vectors and S_cc
  const double bs = double(c.ex_nb) * (4 + double(c.D) * c.D * double(sizeof(T))) +
                    double(c.Ca) * (8 + double(c.D) * (c.D + 1) / 2 * 8 + 3 * c.D * 8 + 8);
  const int G = lanes_per_point(c);
  P3<T>* zq = static_cast<P3<T>*>(c.zq);
  st = pcg_batches(c, max_iters, [&](int it0, int it1) {
    for (int it = it0; it < it1; ++it) {
      if (expl) {
        c.timed("schur_spmv", bs, it, [&] {
          launch_schur_spmv<T>(s, c.D, c.Ca, c.ex_row_ptr, c.ex_bkey,
                               static_cast<const T*>(c.ex_sblk), c.ex_scc, c.u, c.wv, nslot,
                               c.part, c.pcg);
        });
      } else {
        c.timed("schur_point", bp, it, [&] {
          launch_schur_point<T>(s, adj, c.D, G, m, cp, om, mvt, static_cast<const T*>(c.Vinv),
                                zq, c.pcg, c.dl);
        });
        c.timed("schur_cam", bc, it, [&] {
          launch_schur_cam<T>(s, adj, c.D, m, cp, om, c.u, zq, items, nslot, c.part, c.pcg,
                              c.dl);
        });
      }
      c.timed("pcg_update", bu, it, [&] {
        launch_pcg_update<T>(s, c.D, c.Ca, it, c.Minv, Ustar, c.item_off, c.it_count, nslot,
                             c.part, c.dots, c.x, c.r, c.u, c.p, c.sv, c.wv, mvt, c.pcg);
      });
    }
  }, defer);
  *out_state = st;
  return st.matvecs;
}

// |b - S x| / |b| of the PCG solution in c.x (the LM system): one more pass of the matvec
// kernels on x itself, outside the iteration's statistics.
template <typename T>
double true_residual(ba_ctx& c) {
  if (c.Ca == 0) return 0.0;
  hipStream_t s = c.stream;
  const Model m = c.model();
  Compact<T> cp = compact_view<T>(c);
  ObsMetric<T> om = metric_view<T>(c);
  const int nslot = c.it_nslot;   // the items of the solve that produced x
  P3<T>* zq = static_cast<P3<T>*>(c.zq);
  launch_x_to_mv<T>(s, c.D, c.Ca, c.x, c.mvt, c.pcg_diag);
  launch_schur_point<T>(s, false, c.D, lanes_per_point(c), m, cp, om, c.mvt,
                        static_cast<const T*>(c.Vinv), zq, c.pcg_diag, c.dl);
  launch_schur_cam<T>(s, false, c.D, m, cp, om, c.x, zq, items_view(c), nslot, c.part,
                      c.pcg_diag, c.dl);
  launch_true_residual<T>(s, c.D, c.Ca, c.x, c.b, static_cast<const T*>(c.Ustar), c.item_off,
                          nslot, c.part, c.diag);
  HIP_LAUNCH_CHECK();
  HIP_CHECK(hipMemcpyAsync(c.h_pin + 16, c.diag, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  c.sync();
  const double rr = c.h_pin[16], bb = c.h_pin[17];
  return bb > 0 ? std::sqrt(std::max(0.0, rr) / bb) : 0.0;
}

template <typename T>
// The point step of the solve: the PCG point pass run once more on x (the camera step) gives
// z = V*^-1 sum_k W_k^T x_c per point, and dp = hp - z with hp = V*^-1 b_p from the damping
// setup, whose b_p (rhs_p, or -g_p) is the one this step's setup_system used.
void backsub(ba_ctx& c, bool adj) {
  hipStream_t s = c.stream;
  const Model m = c.model();
  Compact<T> cp = compact_view<T>(c);
  ObsMetric<T> om = metric_view<T>(c);
  P3<T>* zq = static_cast<P3<T>*>(c.zq);
  const bool use_z = c.Ca > 0;
  c.timed_multi("backsub", bytes_schur_point(c) + double(c.Pa) * 48, [&] {
    if (use_z) {
      launch_x_to_mv<T>(s, c.D, c.Ca, c.x, c.mvt, c.pcg_diag);
      launch_schur_point<T>(s, adj, c.D, lanes_per_point(c), m, cp, om, c.mvt,
                            static_cast<const T*>(c.Vinv), zq, c.pcg_diag, c.dl);
    }
    launch_backsub<T>(s, c.Pa, c.hp, zq, use_z, c.dp);
  });
}

template <typename T>
ba_status lm_step_impl(ba_ctx& c, ba_step_report* rep) {
  const double t0 = now_ms();
  c.lam = std::max(c.lam, lambda_floor(c));
  ba_step_report R;
  std::memset(&R, 0, sizeof(R));
  R.pcg_true_residual = -1.0;
  R.lambda = c.lam;
  hipStream_t s = c.stream;
  const Model m = c.model();
  const double ts = double(sizeof(T));
  double t_ext = 0, t_lin = 0, t_setup = 0, t_pcg = 0, t_cand = 0;

  if (!c.lin_valid) {
    double ta = now_ms();
    extract(c);
    t_ext = now_ms() - ta;
    R.relinearized = 1;
    if (c.Nh == 0) {
      c.flush_timing(0);
      R.status = BA_EMPTY;
      R.fixpoint_rounds = c.rounds;
      R.ms_extract = t_ext;
      R.ms_total = now_ms() - t0;
      c.step_valid = false;
      c.blocks_valid = false;
      if (rep) *rep = R;
      return BA_EMPTY;
    }
    ta = now_ms();
    linearize<T>(c, false);
    if (explicit_solver(c)) build_schur_pattern<T>(c);
    if (c.opt.timing) c.sync();   // phase times only; the stream orders the work
    t_lin = now_ms() - ta;
    c.lin_valid = true;
  }
  R.fixpoint_rounds = c.rounds;
  R.n_cams_active = c.Ca;
  R.n_points_active = c.Pa;
  R.n_obs_active = c.Nh;

  double ta = now_ms();
  setup_system<T>(c, false, c.lam, nullptr, nullptr);
  if (explicit_solver(c)) assemble_schur_blocks<T>(c);
  if (c.opt.timing) c.sync();
  t_setup = now_ms() - ta;
  c.blocks_valid = true;

  ta = now_ms();
  PcgState st{};
  // the final PCG state is read with the candidate's scalars (no wait between the solve and
  // the back-substitution), except when timing
  c.pcg_pending = -1;
  int iters = run_pcg<T>(c, false, c.opt.pcg_rel_tol, c.opt.pcg_max_iters, &st, !c.opt.timing);
  t_pcg = now_ms() - ta;
  if (c.opt.timing && !explicit_solver(c)) R.pcg_true_residual = true_residual<T>(c);

  ta = now_ms();
  backsub<T>(c, false);
  c.timed("cam_candidate", double(c.Ca + c.n_fixed) * (56 + 120 + 56 + 120) + double(c.Ca) * 48,
          -1, [&] {
            launch_cam_candidate(s, c.Ca, c.n_fixed, c.D, c.cam_src, c.x, c.d_cams, c.camd_hat,
                                 c.d_cand_cams, c.d_cand_tab);
          });
  Compact<T> cp = compact_view<T>(c);
  int nb = 0;
  c.timed("point_candidate",
          double(c.Nh) * (4 + 8 + 4 + ts) + double(c.Pa) * (4 + 24 * 4) + double(c.C) * 240, -1,
          [&] {
            nb = launch_point_candidate<T>(s, m, cp, c.D, c.d_cand_tab, c.x, c.dp, c.gp,
                                           static_cast<const T*>(c.w), c.Xcand, c.partials,
                                           c.dl);
          });
  // scal[4..] = decrease, quad, g_p.dp, bad, cost', g_c.x, max |g_c|
  launch_reduce_partials(s, nb, 5, c.partials, 0x0u, c.D * c.Ca, c.gc, c.x, c.scal + 4);
  HIP_LAUNCH_CHECK();
  HIP_CHECK(hipMemcpyAsync(c.h_pin, c.scal, 11 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(c.h_pin + 11, c.flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  c.sync();
  if (c.pcg_pending >= 0) {   // the solve's last state, copied before the sync
    std::memcpy(&st, pcg_slot(c, c.pcg_pending), sizeof(PcgState));
    iters = st.matvecs;
    c.pcg_pending = -1;
  }
  R.pcg_iters = st.iter;
  R.pcg_breakdown = st.breakdown;
  R.pcg_rel_residual = st.bb > 0 ? std::sqrt(std::max(0.0, st.rr) / st.bb) : 0.0;
  double sc[11];
  std::memcpy(sc, c.h_pin, sizeof(sc));
  int damp_bad = 0;
  std::memcpy(&damp_bad, c.h_pin + 11, sizeof(int));
  const double F = sc[0];
  R.cost_before = F;
  R.rms_px = std::sqrt(sc[1] / double(c.Nh));
  const bool finite_c = !(sc[7] > 0) && std::isfinite(sc[8]);
  const double dF = sc[4];   // actual reduction, summed per observation
  c.last_decrease = dF;
  // reported as F - dF, consistent with the acceptance test (the candidate's own sum, sc[8],
  // carries the rounding of a full cost evaluation)
  const double Fc = finite_c ? F - dF : std::numeric_limits<double>::infinity();
  R.cost_after = Fc;
  const double model = -(sc[6] + sc[9] + 0.5 * sc[5]);
  R.model_decrease = model;
  // max |g| over the compact parameters: points from the linearisation, cameras from gc
  R.grad_inf = std::max(sc[2], c.Ca > 0 ? sc[10] : 0.0);
  if (!std::isfinite(F)) {
    c.flush_timing(iters);
    R.ms_total = now_ms() - t0;
    if (rep) *rep = R;
    throw BaError{BA_ERR_NUMERIC, "non-finite cost at the current parameters"};
  }
  const double ratio = (model > 0 && finite_c) ? dF / model
                                               : -std::numeric_limits<double>::infinity();
  R.gain_ratio = ratio;
  const bool ok = finite_c && dF > 0 && ratio > c.opt.accept_ratio && !st.breakdown && !damp_bad;
  R.accepted = ok ? 1 : 0;
  c.step_valid = true;
  if (ok) {
    c.timed("scatter", double(c.Pa) * 52 + double(c.C) * 60, -1, [&] {
      launch_scatter(s, c.Pa, c.Ca, c.pt_src, c.Xcand, c.cam_src, c.d_cand_cams, c.d_cand_tab,
                     c.d_pts, c.d_cams, c.D == 7 ? c.d_intr : nullptr);
    });
    c.lin_valid = false;
    const double f = std::max(1.0 / 3.0, 1.0 - std::pow(2.0 * ratio - 1.0, 3));
    c.lam = std::max(lambda_floor(c), std::min(c.opt.lambda_max, c.lam * f));
    c.nu = 2.0;
  } else {
    c.lam = std::min(c.lam * c.nu, c.opt.lambda_max);
    c.nu *= 2.0;
  }
  c.sync();
  t_cand = now_ms() - ta;
  c.flush_timing(iters);
  R.ms_extract = t_ext;
  R.ms_linearize = t_lin;
  R.ms_setup = t_setup;
  R.ms_pcg = t_pcg;
  R.ms_candidate = t_cand;
  R.ms_total = now_ms() - t0;
  if (rep) *rep = R;
  return BA_OK;
}

ba_status lm_step_dispatch(ba_ctx& c, ba_step_report* rep) {
  if (!c.have_obs) throw BaError{BA_ERR_STATE, "ba_set_observations has not been called"};
  return c.opt.precision == BA_PRECISION_FP64 ? lm_step_impl<double>(c, rep)
                                              : lm_step_impl<float>(c, rep);
}

// ------------------------------------------------------------------ global positioning
void ensure_gp_buffers(ba_ctx& c) {
  if (c.gp_s) return;
  const size_t ts = c.tsize(), N = size_t(c.N);
  c.gp_s = c.obs.alloc<double>(N);
  c.gp_scand = c.obs.alloc<double>(N);
  c.gp_lin_pm = c.obs.alloc<char>(8 * ts * N);
  c.gp_lin_cm = c.obs.alloc<char>(8 * ts * N);
  c.gp_a_pm = c.obs.alloc<char>(4 * ts * N);
  c.gp_a_cm = c.obs.alloc<char>(4 * ts * N);
}

// Free scales at the inverse distance of the current estimate, pinned ones from the priors;
// the GP damping restarts.
void gp_init(ba_ctx& c) {
  ensure_gp_buffers(c);
  hipStream_t s = c.stream;
  launch_cam_table(s, c.C, c.d_cams, c.d_intr, c.d_camd, c.d_camf);
  HIP_LAUNCH_CHECK();
  launch_gp_init_scales(s, c.N, c.pm_cam, c.pm_pt, c.pm_orig, c.pm_xy, c.pm_depth, c.d_pts,
                        c.d_camd, c.gp_s);
  HIP_LAUNCH_CHECK();
  c.gp_lam = c.opt.lambda_init;
  c.gp_nu = 2.0;
  c.gp_ready = true;
  c.gp_lin_valid = false;
}

// PCG on the camera-centre Schur complement (D = 3); returns the number of matvecs.
template <typename T>
int gp_run_pcg(ba_ctx& c, PcgState* out_state) {
  hipStream_t s = c.stream;
  Compact<T> cp = compact_view<T>(c);
  PcgState st{};
  if (c.Ca == 0) {
    *out_state = st;
    out_state->done = 1;
    return 0;
  }
  const T* Ustar = static_cast<const T*>(c.Ustar);
  int K = 0, nch = 0;
  cam_chunking(c.Nc, K, nch);
  const int nslot = ensure_items(c, 1, K, nch);   // z per camera-major position: no ranges
  resolve_items(c);
  launch_pcg_init<T>(s, 3, c.Ca, c.b, c.Minv, Ustar, c.x, c.r, c.u, c.p, c.sv, c.wv, c.dots,
                     c.mvt, c.pcg, c.opt.pcg_rel_tol * c.opt.pcg_rel_tol, c.opt.pcg_max_iters);
  HIP_LAUNCH_CHECK();
  const CamItems items = items_view(c);
  HIP_LAUNCH_CHECK();
  const double ts = double(sizeof(T));
  const int G = lanes_per_point(c);
  const V4<T>* a_pm = static_cast<const V4<T>*>(c.gp_a_pm);
  const V4<T>* a_cm = static_cast<const V4<T>*>(c.gp_a_cm);
  P3<T>* zq = static_cast<P3<T>*>(c.zq);
  // per observation: slot, A record, camera-major position and z written; per point offset
  // and Vinv; per camera its record
  const double bp = double(c.Nh) * (4 + 4 * ts) + double(c.Nc) * (4 + 3 * ts) +
                    double(c.Pa) * (4 + 6 * ts) + double(c.Ca) * 4 * ts;
  const double bc = double(c.Nc) * 7 * ts + double(c.Ca) * (8 + 24) + double(nslot) * 32;
  const double bu = double(c.Ca) * (48 + 4 + 48 + 6 * ts + 288 + 3 * ts) + double(nslot) * 32;
  st = pcg_batches(c, c.opt.pcg_max_iters, [&](int it0, int it1) {
    for (int it = it0; it < it1; ++it) {
      c.timed("gp_schur_point", bp, it, [&] {
        launch_gp_schur_point<T>(s, G, cp, a_pm, c.mvt, static_cast<const T*>(c.Vinv), zq,
                                 c.pcg, c.dl);
      });
      c.timed("gp_schur_cam", bc, it, [&] {
        launch_gp_schur_cam<T>(s, cp, a_cm, c.u, zq, items, nslot, c.part, c.pcg, c.dl);
      });
      c.timed("gp_pcg_update", bu, it, [&] {
        launch_pcg_update<T>(s, 3, c.Ca, it, c.Minv, Ustar, c.item_off, c.it_count, nslot,
                             c.part, c.dots, c.x, c.r, c.u, c.p, c.sv, c.wv, c.mvt, c.pcg);
      });
    }
  });
  *out_state = st;
  return st.matvecs;
}

template <typename T>
ba_status gp_step_impl(ba_ctx& c, ba_step_report* rep) {
  const double t0 = now_ms();
  ba_step_report R;
  std::memset(&R, 0, sizeof(R));
  R.pcg_true_residual = -1.0;
  if (!c.gp_ready) gp_init(c);
  c.gp_lam = std::max(c.gp_lam, lambda_floor(c));
  R.lambda = c.gp_lam;
  hipStream_t s = c.stream;
  const double ts = double(sizeof(T));
  const double lam = c.gp_lam, dmin = c.opt.diag_min, dmax = c.opt.diag_max;
  const double delta = c.opt.gp_huber;
  Compact<T> cp;
  GpLin<T>* lin_pm = static_cast<GpLin<T>*>(c.gp_lin_pm);
  GpLin<T>* lin_cm = static_cast<GpLin<T>*>(c.gp_lin_cm);
  V4<T>* a_pm = static_cast<V4<T>*>(c.gp_a_pm);
  V4<T>* a_cm = static_cast<V4<T>*>(c.gp_a_cm);
  double ta = now_ms();
  if (!c.gp_lin_valid) {
    extract(c, true);
    // the compaction buffers now hold the GP active sets: the BA step must extract again
    c.lin_valid = false;
    c.step_valid = c.blocks_valid = false;
    R.ms_extract = now_ms() - ta;
    R.relinearized = 1;
    if (c.Nh == 0) {
      c.flush_timing(0);
      R.status = BA_EMPTY;
      R.fixpoint_rounds = c.rounds;
      R.ms_total = now_ms() - t0;
      if (rep) *rep = R;
      return BA_EMPTY;
    }
    cp = compact_view<T>(c);
    ta = now_ms();
    int nbl = 0;
    c.timed("gp_lin", double(c.Nh) * (4 + 8 + 4 + 4 + 8 + 8 * ts) + double(c.Nc) * 8 * ts +
                          double(c.Pa) * (4 + 24 + 24) + double(c.C) * 120,
            -1, [&] {
              nbl = launch_gp_lin<T>(s, lanes_per_point(c), cp, c.orig_hat, c.gp_s, delta,
                                     lin_pm, lin_cm, c.gp, c.partials, c.dl);
            });
    launch_reduce_partials(s, nbl, 3, c.partials, 0x4u, 0, nullptr, nullptr, c.scal);
    HIP_LAUNCH_CHECK();
    R.ms_linearize = now_ms() - ta;
    c.gp_lin_valid = true;
  }
  cp = compact_view<T>(c);
  const int G = lanes_per_point(c);
  R.fixpoint_rounds = c.rounds;
  R.n_cams_active = c.Ca;
  R.n_points_active = c.Pa;
  R.n_obs_active = c.Nh;
  ta = now_ms();
  HIP_CHECK(hipMemsetAsync(c.flags + 1, 0, sizeof(int), s));
  c.timed("gp_point_setup", double(c.Nh) * (8 * ts + 4 + 4 * ts) + double(c.Nc) * 4 * ts +
                                double(c.Pa) * (4 + 6 * ts + 24 + double(sizeof(PtRec<T>))),
          -1, [&] {
            launch_gp_point_setup<T>(s, G, cp, lam, dmin, dmax, lin_pm, a_pm, a_cm,
                                     static_cast<T*>(c.Vinv), c.hp,
                                     static_cast<PtRec<T>*>(c.prec), c.flags + 1);
          });
  c.timed("gp_cam_assemble",
          double(c.Nc) * (4 + 12 * ts) + double(c.Pa) * double(sizeof(PtRec<T>)) +
              double(c.Ca) * (8 + 6 * ts + 6 * 8 + 6 * 8),
          -1, [&] {
            launch_gp_cam_assemble<T>(s, cp, lam, dmin, dmax, lin_cm, a_cm,
                                      static_cast<const PtRec<T>*>(c.prec),
                                      static_cast<T*>(c.Ustar), c.gc, c.b, c.Minv);
          });
  HIP_LAUNCH_CHECK();
  R.ms_setup = now_ms() - ta;
  ta = now_ms();
  PcgState st{};
  const int iters = gp_run_pcg<T>(c, &st);
  R.pcg_iters = st.iter;
  R.pcg_breakdown = st.breakdown;
  R.pcg_rel_residual = st.bb > 0 ? std::sqrt(std::max(0.0, st.rr) / st.bb) : 0.0;
  R.ms_pcg = now_ms() - ta;
  ta = now_ms();
  c.timed("gp_backsub", double(c.Nh) * (4 + 4 * ts) + double(c.Pa) * (4 + 6 * ts + 48) +
                            double(c.Ca) * 24,
          -1, [&] {
            launch_gp_backsub<T>(s, G, cp, a_pm, static_cast<const T*>(c.Vinv), c.hp, c.x, c.dp);
          });
  int nb = 0;
  c.timed("gp_candidate", double(c.Nh) * (4 + 8 + 4 + 4 + 8 + 8) + double(c.Pa) * (4 + 24 * 4) +
                              double(c.C) * 240,
          -1, [&] {
            nb = launch_gp_candidate<T>(s, lanes_per_point(c), cp, c.orig_hat, c.gp_s, delta,
                                        lam, dmin, dmax, c.x, c.dp, c.gp, c.Xcand, c.gp_scand,
                                        c.partials, c.dl);
          });
  // scal[4..] = decrease, quad, g_X.dX + g_s.ds, bad, cost', g_c.dc, max |g_c|
  launch_reduce_partials(s, nb, 5, c.partials, 0x0u, 3 * c.Ca, c.gc, c.x, c.scal + 4);
  HIP_LAUNCH_CHECK();
  HIP_CHECK(hipMemcpyAsync(c.h_pin, c.scal, 11 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(c.h_pin + 11, c.flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  c.sync();
  double sc[11];
  std::memcpy(sc, c.h_pin, sizeof(sc));
  int damp_bad = 0;
  std::memcpy(&damp_bad, c.h_pin + 11, sizeof(int));
  const double F = sc[0];
  R.cost_before = F;
  R.rms_px = std::sqrt(sc[1] / double(c.Nh));
  const bool finite_c = !(sc[7] > 0) && std::isfinite(sc[8]);
  const double dF = sc[4];
  c.gp_last_decrease = dF;
  R.cost_after = finite_c ? F - dF : std::numeric_limits<double>::infinity();
  const double model = -(sc[6] + sc[9] + 0.5 * sc[5]);
  R.model_decrease = model;
  R.grad_inf = std::max(sc[2], c.Ca > 0 ? sc[10] : 0.0);
  if (!std::isfinite(F)) {
    c.flush_timing(iters);
    R.ms_total = now_ms() - t0;
    if (rep) *rep = R;
    throw BaError{BA_ERR_NUMERIC, "non-finite GP cost at the current parameters"};
  }
  const double ratio = (model > 0 && finite_c) ? dF / model
                                               : -std::numeric_limits<double>::infinity();
  R.gain_ratio = ratio;
  const bool ok = finite_c && dF > 0 && ratio > c.opt.accept_ratio && !st.breakdown && !damp_bad;
  R.accepted = ok ? 1 : 0;
  if (ok) {
    c.timed("gp_scatter", double(c.Pa) * 52 + double(c.Ca) * 60 + double(c.Nh) * 16, -1, [&] {
      launch_gp_scatter(s, c.Pa, c.Ca, c.Nh, c.pt_src, c.Xcand, c.cam_src, c.x, c.depth_hat,
                        c.orig_hat, c.gp_scand, c.d_pts, c.d_cams, c.gp_s);
    });
    c.gp_lin_valid = false;
    const double f = std::max(1.0 / 3.0, 1.0 - std::pow(2.0 * ratio - 1.0, 3));
    c.gp_lam = std::max(lambda_floor(c), std::min(c.opt.lambda_max, c.gp_lam * f));
    c.gp_nu = 2.0;
  } else {
    c.gp_lam = std::min(c.gp_lam * c.gp_nu, c.opt.lambda_max);
    c.gp_nu *= 2.0;
  }
  c.sync();
  R.ms_candidate = now_ms() - ta;
  c.flush_timing(iters);
  R.ms_total = now_ms() - t0;
  if (rep) *rep = R;
  return BA_OK;
}

ba_status gp_step_dispatch(ba_ctx& c, ba_step_report* rep) {
  if (!c.have_obs) throw BaError{BA_ERR_STATE, "ba_set_observations has not been called"};
  return c.opt.precision == BA_PRECISION_FP64 ? gp_step_impl<double>(c, rep)
                                              : gp_step_impl<float>(c, rep);
}

// Returns false when the adjoint PCG stopped at adjoint_max_iters above its tolerance (the
// gradients are still written, from the last iterate); the message is left in c.err.
template <typename T>
bool adjoint_impl(ba_ctx& c, const double* grad_cams, const double* grad_points, float* gxy,
                  float* gdepth) {
  bool converged = true;
  hipStream_t s = c.stream;
  ensure_adjoint_buffers(c);
  // the full Hessian's terms are read by the adjoint-mode kernels while this call runs
  struct CeScope {
    ba_ctx& c;
    CeScope(ba_ctx& cc, bool on) : c(cc) { c.ce_on = on; }
    ~CeScope() { c.ce_on = false; }
  } ce_scope(c, c.opt.adjoint_hessian == BA_ADJOINT_FULL);
  c.to_device(c.grad_cams_d, grad_cams, sizeof(double) * 7 * size_t(c.C));
  c.to_device(c.grad_pts_d, grad_points, sizeof(double) * 3 * size_t(c.P));
  HIP_CHECK(hipMemsetAsync(c.gxy_d, 0, sizeof(float) * 2 * size_t(c.N), s));
  HIP_CHECK(hipMemsetAsync(c.gdepth_d, 0, sizeof(float) * size_t(c.N), s));
  extract(c);
  c.lin_valid = false;   // the LM linearisation buffers are reused below
  c.blocks_valid = false;
  c.step_valid = false;
  if (c.Nh > 0) {
    linearize<T>(c, true);
    launch_adjoint_rhs(s, c.Ca, c.Pa, c.cam_src, c.d_cams, c.grad_cams_d, c.pt_src, c.pt_user_d,
                       c.grad_pts_d, c.rhs_c, c.rhs_p);
    HIP_LAUNCH_CHECK();
    setup_system<T>(c, true, c.opt.adjoint_damping, c.rhs_c, c.rhs_p);
    PcgState st{};
    const double tol = c.opt.adjoint_rel_tol;
    const int maxit = c.opt.adjoint_max_iters;
    const int mv = run_pcg<T>(c, true, tol, maxit, &st);
    backsub<T>(c, true);
    Compact<T> cp = compact_view<T>(c);
    launch_adjoint_obs<T>(s, c.model(), cp, metric_view<T>(c), c.x, c.dp, c.orig_hat, c.gxy_d,
                          c.gdepth_d);
    HIP_LAUNCH_CHECK();
    int bad = 0;
    HIP_CHECK(hipMemcpyAsync(c.h_pin, c.flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    c.sync();
    std::memcpy(&bad, c.h_pin, sizeof(int));
    c.flush_timing(mv);
    if (bad) throw BaError{BA_ERR_NUMERIC, "singular point block in the adjoint system"};
    if (st.breakdown) throw BaError{BA_ERR_NUMERIC, "adjoint PCG broke down"};
    if (!st.done && c.Ca > 0) {
      converged = false;
      char msg[160];
      std::snprintf(msg, sizeof(msg),
                    "adjoint PCG stopped after %d iterations at relative residual %.3e "
                    "(tolerance %.3e)", st.iter, st.bb > 0 ? std::sqrt(st.rr / st.bb) : 0.0, tol);
      c.err = msg;
    }
  }
  c.sync();
  HIP_CHECK(hipMemcpyAsync(gxy, c.gxy_d, sizeof(float) * 2 * size_t(c.N), hipMemcpyDefault, s));
  if (gdepth)
    HIP_CHECK(hipMemcpyAsync(gdepth, c.gdepth_d, sizeof(float) * size_t(c.N), hipMemcpyDefault,
                             s));
  c.sync();
  return converged;
}

// Counting sort by an integer key in [0, K): stable.
void counting_order(const std::vector<int32_t>& key, int K, std::vector<int32_t>& order,
                    std::vector<int32_t>& offsets) {
  offsets.assign(size_t(K) + 1, 0);
  for (int32_t k : key) offsets[size_t(k) + 1]++;
  for (int i = 0; i < K; ++i) offsets[i + 1] += offsets[i];
  std::vector<int32_t> next(offsets.begin(), offsets.end() - 1);
  order.resize(key.size());
  for (size_t i = 0; i < key.size(); ++i) order[next[key[i]]++] = int32_t(i);
}

void points_user_to_internal(ba_ctx& c, const std::vector<double>& user,
                             std::vector<double>& internal) {
  internal.resize(user.size());
  for (int i = 0; i < c.P; ++i)
    for (int k = 0; k < 3; ++k) internal[3 * size_t(i) + k] = user[3 * size_t(c.pt_user[i]) + k];
}

void points_internal_to_user(ba_ctx& c, const std::vector<double>& internal,
                             std::vector<double>& user) {
  user.resize(internal.size());
  for (int i = 0; i < c.P; ++i)
    for (int k = 0; k < 3; ++k) user[3 * size_t(c.pt_user[i]) + k] = internal[3 * size_t(i) + k];
}

// Where ba_lm_step_noalloc puts each per-step buffer inside the static scratch array (the
// sizes the context allocates for the same buffers, each slice aligned to 256 bytes).
struct ScratchPlan {
  size_t flags = 0, pcg = 0, pcg_diag = 0, diag = 0, partials = 0, dots = 0, part = 0,
         item_off = 0, item_at = 0, rb = 0, scan = 0, total = 0;
};

ScratchPlan plan_scratch(const ba_ctx& c) {
  ScratchPlan p;
  auto take = [&](size_t bytes) {
    const size_t o = p.total;
    p.total += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t C = size_t(c.C), nd = size_t(c.D);
  p.flags = take(4 * sizeof(int));
  p.pcg = take(sizeof(PcgState));
  p.pcg_diag = take(sizeof(PcgState));
  p.diag = take(4 * sizeof(double));
  p.partials = take(5 * (size_t(c.P) * 16 / kBlock + 16) * sizeof(double));
  p.dots = take(2 * 3 * C * sizeof(double));
  p.part = take(part_rows(c.D) * item_slots(c.C) * sizeof(double));
  p.item_off = take((C + 2) * sizeof(int));
  p.item_at = take(kMaxRanges * (C + kCamChunks) * sizeof(int4));
  p.rb = take(kMaxRanges * C * sizeof(int));
  p.scan = take(c.scan_temp_size);
  return p;
}

// Points the context's per-step buffers into the scratch array for one call and restores
// them afterwards (also when the step throws).
struct ScratchSwap {
  ba_ctx& c;
  int* flags;
  PcgState *pcg, *pcg_diag;
  double *diag, *partials, *dots, *part;
  int *item_off, *rb;
  int4* item_at;
  void* scan;
  ScratchSwap(ba_ctx& cc, char* base, const ScratchPlan& p)
      : c(cc), flags(cc.flags), pcg(cc.pcg), pcg_diag(cc.pcg_diag), diag(cc.diag),
        partials(cc.partials), dots(cc.dots), part(cc.part), item_off(cc.item_off),
        rb(cc.rb), item_at(cc.item_at), scan(cc.scan_temp) {
    c.items_ok = false;   // the items live in the buffers being swapped
    settle_items();
    c.flags = reinterpret_cast<int*>(base + p.flags);
    c.pcg = reinterpret_cast<PcgState*>(base + p.pcg);
    c.pcg_diag = reinterpret_cast<PcgState*>(base + p.pcg_diag);
    c.diag = reinterpret_cast<double*>(base + p.diag);
    c.partials = reinterpret_cast<double*>(base + p.partials);
    c.dots = reinterpret_cast<double*>(base + p.dots);
    c.part = reinterpret_cast<double*>(base + p.part);
    c.item_off = reinterpret_cast<int*>(base + p.item_off);
    c.item_at = reinterpret_cast<int4*>(base + p.item_at);
    c.rb = reinterpret_cast<int*>(base + p.rb);
    c.scan_temp = base + p.scan;
  }
  ~ScratchSwap() {
    c.flags = flags;
    c.pcg = pcg;
    c.pcg_diag = pcg_diag;
    c.diag = diag;
    c.partials = partials;
    c.dots = dots;
    c.part = part;
    c.item_off = item_off;
    c.item_at = item_at;
    c.rb = rb;
    c.scan_temp = scan;
    c.items_ok = false;
    settle_items();
  }
  // a pending item-count copy reads the buffers being swapped: let it land (the counts are
  // rebuilt with the items)
  void settle_items() {
    if (c.items_pending) (void)hipEventSynchronize(c.items_ev);
    c.items_pending = false;
  }
  ScratchSwap(const ScratchSwap&) = delete;
  ScratchSwap& operator=(const ScratchSwap&) = delete;
};

}  // namespace

// ================================================================== C ABI
extern "C" {

void ba_default_options(ba_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = BA_PRECISION_MIXED;
  o->img_w = 640;
  o->img_h = 480;
  o->activity_rule = BA_ACTIVITY_ROWS;
  o->min_depth = 0.1;
  o->huber_px = 0.0;
  o->filter_px = 0.0;
  o->lambda_init = 1e-3;
  o->lambda_min = 1e-12;
  o->lambda_max = 1e12;
  o->diag_min = 1e-6;
  o->diag_max = 1e32;
  o->accept_ratio = 1e-3;
  o->pcg_max_iters = 100;
  o->pcg_check_every = 8;
  o->pcg_rel_tol = 1e-6;
  o->cost_rel_tol = 1e-10;
  o->grad_tol = 1e-10;
  o->max_lm_iters = 100;
  o->timing = 0;
  o->adjoint_max_iters = 5000;
  o->adjoint_damping = 0.0;
  o->refine_focal = 0;
  o->gp_huber = 0.1;
  o->solver = BA_SOLVER_IMPLICIT;
  o->adjoint_hessian = BA_ADJOINT_FULL;
  o->adjoint_rel_tol = 1e-10;
  o->hip_stream = nullptr;
}

ba_status ba_create(const ba_options* opt, int32_t n_cams, int32_t n_points, const double* cams,
                    const double* intr, const double* points, ba_ctx** out) {
  g_create_error.clear();
  if (!out) {
    g_create_error = "out is NULL";
    return BA_ERR_ARG;
  }
  *out = nullptr;
  ba_options o;
  if (opt)
    o = *opt;
  else
    ba_default_options(&o);
  if (n_cams < 1 || n_points < 1 || n_cams > kMaxCams || n_points > kMaxPoints || !cams ||
      !intr || !points) {
    g_create_error = "need 1 <= n_cams <= 2^27 - 1, 1 <= n_points <= 2^27 - 1 and non-NULL "
                     "cams, intr, points";
    return BA_ERR_ARG;
  }
  if ((o.precision != BA_PRECISION_FP64 && o.precision != BA_PRECISION_MIXED) ||
      (o.activity_rule != BA_ACTIVITY_ROWS && o.activity_rule != BA_ACTIVITY_LITERAL) ||
      o.img_w <= 0 || o.img_h <= 0 || !(o.lambda_min > 0) || !(o.lambda_max >= o.lambda_min) ||
      !(o.lambda_init > 0) || o.pcg_max_iters < 0 || !(o.pcg_rel_tol >= 0) ||
      !(o.diag_min > 0) || !(o.diag_max >= o.diag_min) || o.adjoint_max_iters < 0 ||
      !(o.adjoint_damping >= 0) || (o.refine_focal != 0 && o.refine_focal != 1) ||
      !std::isfinite(o.gp_huber) ||
      (o.solver != BA_SOLVER_IMPLICIT && o.solver != BA_SOLVER_EXPLICIT) ||
      (o.adjoint_hessian != BA_ADJOINT_FULL && o.adjoint_hessian != BA_ADJOINT_GAUSS_NEWTON) ||
      !(o.adjoint_rel_tol >= 0)) {
    g_create_error = "invalid options";
    return BA_ERR_ARG;
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    g_create_error = "no HIP device available";
    return BA_ERR_DEVICE;
  }
  ba_ctx* c = new (std::nothrow) ba_ctx();
  if (!c) {
    g_create_error = "host allocation failed";
    return BA_ERR_OOM;
  }
  c->opt = o;
  c->D = o.refine_focal ? 7 : 6;
  c->C = n_cams;
  c->P = n_points;
  c->lam = o.lambda_init;
  try {
    if (o.hip_stream) {
      c->stream = static_cast<hipStream_t>(o.hip_stream);
    } else {
      HIP_CHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&c->h_pin), 64 * sizeof(double)));
    for (auto& e : c->pcg_ev) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&c->items_ev, hipEventDisableTiming));
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    c->device = dev;
    c->scratch_dev = scratch_address(dev);
    HIP_CHECK(hipDeviceGetAttribute(&c->dl.n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_CHECK(hipDeviceGetAttribute(&c->dl.lds_per_block,
                                    hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    Arena& A = c->par;
    c->d_cams = A.alloc<double>(7 * size_t(n_cams));
    c->d_intr = A.alloc<double>(3 * size_t(n_cams));
    c->d_pts = A.alloc<double>(3 * size_t(n_points));
    c->d_fixed = A.alloc<uint8_t>(n_cams);
    c->d_fixed_rank = A.alloc<int>(n_cams);
    c->d_camd = A.alloc<Cam<double>>(n_cams);
    c->d_camf = A.alloc<Cam<float>>(n_cams);
    c->d_cand_tab = A.alloc<Cam<double>>(n_cams);
    c->d_cand_cams = A.alloc<double>(7 * size_t(n_cams));
    std::vector<double> hc, hi, hpnt;
    fetch(*c, hc, cams, 7 * size_t(n_cams));
    fetch(*c, hi, intr, 3 * size_t(n_cams));
    fetch(*c, hpnt, points, 3 * size_t(n_points));
    for (double v : hc)
      if (!std::isfinite(v)) throw BaError{BA_ERR_ARG, "non-finite camera parameter"};
    for (double v : hpnt)
      if (!std::isfinite(v)) throw BaError{BA_ERR_ARG, "non-finite point"};
    for (int i = 0; i < n_cams; ++i) {
      const double* q = &hc[7 * size_t(i)];
      if (!(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3] > 0))
        throw BaError{BA_ERR_ARG, "zero quaternion"};
      if (!(hi[3 * size_t(i)] > 0)) throw BaError{BA_ERR_ARG, "focal length must be > 0"};
    }
    c->pt_user.resize(n_points);
    c->pt_internal.resize(n_points);
    for (int i = 0; i < n_points; ++i) c->pt_user[i] = c->pt_internal[i] = i;
    c->fixed_h.assign(n_cams, 0);
    store(*c, c->d_cams, hc.data(), hc.size());
    store(*c, c->d_intr, hi.data(), hi.size());
    store(*c, c->d_pts, hpnt.data(), hpnt.size());
    store(*c, c->d_fixed, c->fixed_h.data(), c->fixed_h.size());
    std::vector<int32_t> fr(size_t(n_cams), -1);
    store(*c, c->d_fixed_rank, fr.data(), fr.size());
  } catch (const BaError& err) {
    g_create_error = err.msg;
    delete c;
    return err.code;
  }
  *out = c;
  return BA_OK;
}

ba_status ba_set_observations(ba_ctx* c, int64_t n_obs, const int32_t* cam_idx,
                              const int32_t* pt_idx, const float* xy) {
  return guarded(c, [&]() -> ba_status {
    if (n_obs < 0 || n_obs > kMaxObs)
      return fail(c, BA_ERR_ARG, "n_obs must be in [0, 2^29 - 1]");
    if (n_obs > 0 && (!cam_idx || !pt_idx || !xy))
      return fail(c, BA_ERR_ARG, "NULL observation array");
    std::vector<int32_t> hc, hp;
    std::vector<float> hxy;
    fetch(*c, hc, cam_idx, size_t(n_obs));
    fetch(*c, hp, pt_idx, size_t(n_obs));
    fetch(*c, hxy, xy, 2 * size_t(n_obs));
    for (int64_t k = 0; k < n_obs; ++k) {
      if (hc[k] < 0 || hc[k] >= c->C)
        return fail(c, BA_ERR_ARG, "camera index out of range at observation " + std::to_string(k));
      if (hp[k] < 0 || hp[k] >= c->P)
        return fail(c, BA_ERR_ARG, "point index out of range at observation " + std::to_string(k));
    }
    // current points back to caller order before renumbering
    std::vector<double> pts_int, pts_user;
    download(*c, pts_int, c->d_pts, 3 * size_t(c->P));
    points_internal_to_user(*c, pts_int, pts_user);

    // internal point order: by smallest observing camera (points seen by the same cameras
    // become neighbours, which keeps the camera-major gathers local), stable
    const int C = c->C, P = c->P;
    std::vector<int32_t> key(P, C);
    for (int64_t k = 0; k < n_obs; ++k) key[hp[k]] = std::min(key[hp[k]], hc[k]);
    std::vector<int32_t> order, offs;
    counting_order(key, C + 1, order, offs);
    c->pt_user = order;                       // internal -> caller
    for (int i = 0; i < P; ++i) c->pt_internal[order[i]] = i;
    // point-major observation order (stable in the caller's order within a point)
    std::vector<int32_t> pint(n_obs);
    for (int64_t k = 0; k < n_obs; ++k) pint[k] = c->pt_internal[hp[k]];
    std::vector<int32_t> pm_order, pt_off;
    counting_order(pint, P, pm_order, pt_off);
    std::vector<int32_t> pm_cam(n_obs), pm_pt(n_obs);
    std::vector<float> pm_xy(2 * size_t(n_obs));
    for (int64_t j = 0; j < n_obs; ++j) {
      const int32_t k = pm_order[j];
      pm_cam[j] = hc[k];
      pm_pt[j] = pint[k];
      pm_xy[2 * j] = hxy[2 * size_t(k)];
      pm_xy[2 * j + 1] = hxy[2 * size_t(k) + 1];
    }
    // camera-major order over the point-major positions (stable: increasing point)
    std::vector<int32_t> cm_perm, cm_off;
    counting_order(pm_cam, C, cm_perm, cm_off);
    std::vector<int32_t> inv_cm(static_cast<size_t>(n_obs)), cm_cam(static_cast<size_t>(n_obs));
    for (int64_t mm = 0; mm < n_obs; ++mm) {
      inv_cm[size_t(cm_perm[size_t(mm)])] = int32_t(mm);
      cm_cam[size_t(mm)] = pm_cam[size_t(cm_perm[size_t(mm)])];
    }

    c->N = n_obs;
    c->have_obs = false;
    alloc_obs_buffers(*c);
    std::vector<float> zeros(size_t(n_obs), 0.0f);
    store(*c, c->pm_cam, pm_cam.data(), pm_cam.size());
    store(*c, c->pm_pt, pm_pt.data(), pm_pt.size());
    store(*c, c->pm_orig, pm_order.data(), pm_order.size());
    store(*c, reinterpret_cast<float*>(c->pm_xy), pm_xy.data(), pm_xy.size());
    store(*c, c->pm_depth, zeros.data(), zeros.size());
    store(*c, c->pt_off, pt_off.data(), pt_off.size());
    store(*c, c->cm_off, cm_off.data(), cm_off.size());
    store(*c, c->inv_cm, inv_cm.data(), inv_cm.size());
    store(*c, c->cm_cam, cm_cam.data(), cm_cam.size());
    store(*c, c->pt_user_d, c->pt_user.data(), c->pt_user.size());
    points_user_to_internal(*c, pts_user, pts_int);
    store(*c, c->d_pts, pts_int.data(), pts_int.size());
    c->pm_orig_h = pm_order;
    c->have_obs = true;
    c->have_priors = false;
    c->lam_d = 0.0;
    c->lam = c->opt.lambda_init;
    c->nu = 2.0;
    c->lin_valid = c->ext_valid = c->step_valid = c->blocks_valid = false;
    c->gp_lin_valid = false;
    return BA_OK;
  });
}

ba_status ba_set_depth_priors(ba_ctx* c, const float* depth, const uint8_t* valid,
                              double lambda_d) {
  return guarded(c, [&]() -> ba_status {
    if (!c->have_obs) return fail(c, BA_ERR_STATE, "set observations before depth priors");
    if (!(lambda_d >= 0) || !std::isfinite(lambda_d))
      return fail(c, BA_ERR_ARG, "lambda_d must be finite and >= 0");
    if (c->N > 0 && !depth) return fail(c, BA_ERR_ARG, "depth is NULL");
    std::vector<float> hd;
    std::vector<uint8_t> hv;
    fetch(*c, hd, depth, size_t(c->N));
    if (valid) fetch(*c, hv, valid, size_t(c->N));
    std::vector<float> pm(size_t(c->N));
    for (int64_t j = 0; j < c->N; ++j) {
      const int32_t k = c->pm_orig_h[j];
      const float d = hd[k];
      const bool ok = (!valid || hv[k] != 0) && std::isfinite(d) && d > 0.0f;
      pm[j] = ok ? d : 0.0f;
    }
    store(*c, c->pm_depth, pm.data(), pm.size());
    c->have_priors = true;
    c->gp_ready = false;   // pinned scales change with the priors
    c->lam_d = lambda_d;
    c->lin_valid = c->ext_valid = c->step_valid = c->blocks_valid = false;
    c->gp_lin_valid = false;
    return BA_OK;
  });
}

ba_status ba_set_fixed_cameras(ba_ctx* c, int32_t n, const int32_t* ids) {
  return guarded(c, [&]() -> ba_status {
    if (n < 0 || (n > 0 && !ids)) return fail(c, BA_ERR_ARG, "invalid fixed camera list");
    std::vector<int32_t> h;
    fetch(*c, h, ids, size_t(n));
    std::vector<uint8_t> f(size_t(c->C), 0);
    for (int32_t i : h) {
      if (i < 0 || i >= c->C) return fail(c, BA_ERR_ARG, "fixed camera index out of range");
      f[i] = 1;
    }
    c->fixed_h = f;
    c->n_fixed = 0;
    std::vector<int32_t> fr(size_t(c->C), -1);
    for (int i = 0; i < c->C; ++i)
      if (f[i]) fr[i] = c->n_fixed++;
    store(*c, c->d_fixed, f.data(), f.size());
    store(*c, c->d_fixed_rank, fr.data(), fr.size());
    c->lin_valid = c->ext_valid = c->step_valid = c->blocks_valid = false;
    c->gp_lin_valid = false;
    return BA_OK;
  });
}

ba_status ba_lm_step(ba_ctx* c, ba_step_report* rep) {
  return guarded(c, [&]() -> ba_status { return lm_step_dispatch(*c, rep); });
}

ba_status ba_lm_step_noalloc(ba_ctx* c, ba_step_report* rep) {
  return guarded(c, [&]() -> ba_status {
    if (!c->have_obs) return fail(c, BA_ERR_STATE, "ba_set_observations has not been called");
    if (c->opt.solver == BA_SOLVER_EXPLICIT)
      return fail(c, BA_ERR_STATE,
                  "ba_lm_step_noalloc: the explicit solver allocates its block pattern");
    if (c->opt.timing)
      return fail(c, BA_ERR_STATE, "ba_lm_step_noalloc: timing creates events; set timing = 0");
    const ScratchPlan p = plan_scratch(*c);
    if (p.total > kScratchBytes)
      return fail(c, BA_ERR_ARG,
                  "ba_lm_step_noalloc: this problem needs " + std::to_string(p.total) +
                      " bytes of step scratch, more than the " + std::to_string(kScratchBytes) +
                      "-byte static array (use ba_lm_step)");
    if (!c->scratch_dev)
      return fail(c, BA_ERR_DEVICE, "ba_lm_step_noalloc: no scratch address on this device");
    ScratchSwap swap(*c, static_cast<char*>(c->scratch_dev), p);
    return lm_step_dispatch(*c, rep);
  });
}

ba_status ba_solve(ba_ctx* c, ba_solve_report* rep) {
  return guarded(c, [&]() -> ba_status {
    const double t0 = now_ms();
    ba_solve_report S;
    std::memset(&S, 0, sizeof(S));
    ba_step_report R;
    ba_status st = BA_OK;
    bool first = true;
    for (int it = 0; it < c->opt.max_lm_iters; ++it) {
      st = lm_step_dispatch(*c, &R);
      S.iterations += 1;
      if (st == BA_EMPTY) {
        S.stop_reason = 4;
        break;
      }
      if (first) {
        S.initial_cost = R.cost_before;
        S.initial_rms_px = R.rms_px;
        first = false;
      }
      S.total_pcg_iters += R.pcg_iters;
      S.accepted += R.accepted;
      S.final_cost = R.accepted ? R.cost_after : R.cost_before;
      S.final_rms_px = R.rms_px;
      if (R.grad_inf <= c->opt.grad_tol) {
        S.stop_reason = 2;
        break;
      }
      if (R.accepted && c->last_decrease <= c->opt.cost_rel_tol * R.cost_before) {
        S.stop_reason = 1;
        break;
      }
      if (!R.accepted && R.lambda >= c->opt.lambda_max) {
        S.stop_reason = 3;
        break;
      }
    }
    S.lambda = c->lam;
    S.ms_total = now_ms() - t0;
    if (rep) *rep = S;
    return st == BA_EMPTY ? BA_EMPTY : BA_OK;
  });
}

ba_status ba_gp_step(ba_ctx* c, ba_step_report* rep) {
  return guarded(c, [&]() -> ba_status { return gp_step_dispatch(*c, rep); });
}

ba_status ba_gp_solve(ba_ctx* c, ba_solve_report* rep) {
  return guarded(c, [&]() -> ba_status {
    const double t0 = now_ms();
    ba_solve_report S;
    std::memset(&S, 0, sizeof(S));
    ba_step_report R;
    ba_status st = BA_OK;
    bool first = true;
    for (int it = 0; it < c->opt.max_lm_iters; ++it) {
      st = gp_step_dispatch(*c, &R);
      S.iterations += 1;
      if (st == BA_EMPTY) {
        S.stop_reason = 4;
        break;
      }
      if (first) {
        S.initial_cost = R.cost_before;
        S.initial_rms_px = R.rms_px;
        first = false;
      }
      S.total_pcg_iters += R.pcg_iters;
      S.accepted += R.accepted;
      S.final_cost = R.accepted ? R.cost_after : R.cost_before;
      S.final_rms_px = R.rms_px;
      if (R.grad_inf <= c->opt.grad_tol) {
        S.stop_reason = 2;
        break;
      }
      if (R.accepted && c->gp_last_decrease <= c->opt.cost_rel_tol * R.cost_before) {
        S.stop_reason = 1;
        break;
      }
      if (!R.accepted && R.lambda >= c->opt.lambda_max) {
        S.stop_reason = 3;
        break;
      }
    }
    S.lambda = c->gp_lam;
    S.ms_total = now_ms() - t0;
    if (rep) *rep = S;
    return st == BA_EMPTY ? BA_EMPTY : BA_OK;
  });
}

ba_status ba_gp_get_scales(const ba_ctx* cc, double* scales) {
  ba_ctx* c = const_cast<ba_ctx*>(cc);
  return guarded(c, [&]() -> ba_status {
    if (!scales) return fail(c, BA_ERR_ARG, "scales is NULL");
    if (!c->have_obs) return fail(c, BA_ERR_STATE, "ba_set_observations has not been called");
    if (!c->gp_ready) gp_init(*c);
    HIP_CHECK(hipMemcpyAsync(scales, c->gp_s, sizeof(double) * size_t(c->N), hipMemcpyDefault,
                             c->stream));
    c->sync();
    return BA_OK;
  });
}

ba_status ba_gp_reset(ba_ctx* c) {
  return guarded(c, [&]() -> ba_status {
    if (!c->have_obs) return fail(c, BA_ERR_STATE, "ba_set_observations has not been called");
    gp_init(*c);
    c->sync();
    return BA_OK;
  });
}

ba_status ba_get_params(const ba_ctx* cc, double* cams, double* points) {
  ba_ctx* c = const_cast<ba_ctx*>(cc);
  return guarded(c, [&]() -> ba_status {
    if (cams) {
      HIP_CHECK(hipMemcpyAsync(cams, c->d_cams, sizeof(double) * 7 * size_t(c->C),
                               hipMemcpyDefault, c->stream));
      c->sync();
    }
    if (points) {
      std::vector<double> in, user;
      download(*c, in, c->d_pts, 3 * size_t(c->P));
      points_internal_to_user(*c, in, user);
      store(*c, points, user.data(), user.size());
    }
    return BA_OK;
  });
}

ba_status ba_get_intrinsics(const ba_ctx* cc, double* intr) {
  ba_ctx* c = const_cast<ba_ctx*>(cc);
  return guarded(c, [&]() -> ba_status {
    if (!intr) return fail(c, BA_ERR_ARG, "intr is NULL");
    HIP_CHECK(hipMemcpyAsync(intr, c->d_intr, sizeof(double) * 3 * size_t(c->C),
                             hipMemcpyDefault, c->stream));
    c->sync();
    return BA_OK;
  });
}

ba_status ba_set_params(ba_ctx* c, const double* cams, const double* points) {
  return guarded(c, [&]() -> ba_status {
    if (cams) {
      std::vector<double> h;
      fetch(*c, h, cams, 7 * size_t(c->C));
      for (double v : h)
        if (!std::isfinite(v)) return fail(c, BA_ERR_ARG, "non-finite camera parameter");
      store(*c, c->d_cams, h.data(), h.size());
    }
    if (points) {
      std::vector<double> h, in;
      fetch(*c, h, points, 3 * size_t(c->P));
      for (double v : h)
        if (!std::isfinite(v)) return fail(c, BA_ERR_ARG, "non-finite point");
      points_user_to_internal(*c, h, in);
      store(*c, c->d_pts, in.data(), in.size());
    }
    c->lam = c->opt.lambda_init;
    c->nu = 2.0;
    c->lin_valid = c->step_valid = c->blocks_valid = false;
    c->gp_ready = c->gp_lin_valid = false;   // free GP scales restart from the new estimate
    return BA_OK;
  });
}

ba_status ba_get_active(const ba_ctx* cc, uint8_t* cams, uint8_t* points, uint8_t* obs) {
  ba_ctx* c = const_cast<ba_ctx*>(cc);
  return guarded(c, [&]() -> ba_status {
    if (!c->ext_valid) return fail(c, BA_ERR_STATE, "no extraction has run yet");
    if (cams) {
      std::vector<uint8_t> h;
      download(*c, h, c->act_c, size_t(c->C));
      store(*c, cams, h.data(), h.size());
    }
    if (points) {
      std::vector<uint8_t> h, u(size_t(c->P));
      download(*c, h, c->act_p, size_t(c->P));
      for (int i = 0; i < c->P; ++i) u[c->pt_user[i]] = h[i];
      store(*c, points, u.data(), u.size());
    }
    if (obs) {
      std::vector<uint8_t> h, u(size_t(c->N));
      download(*c, h, c->vrow, size_t(c->N));
      for (int64_t j = 0; j < c->N; ++j) u[c->pm_orig_h[j]] = h[j] ? 1 : 0;
      store(*c, obs, u.data(), u.size());
    }
    return BA_OK;
  });
}

ba_status ba_get_last_step(const ba_ctx* cc, double* dcams, double* dpoints) {
  ba_ctx* c = const_cast<ba_ctx*>(cc);
  return guarded(c, [&]() -> ba_status {
    if (!c->step_valid) return fail(c, BA_ERR_STATE, "no LM step has been computed");
    std::vector<int> src;
    if (dcams) {
      const size_t D = size_t(c->D);
      std::vector<double> x, out(D * size_t(c->C), 0.0);
      download(*c, x, c->x, D * size_t(c->Ca));
      download(*c, src, c->cam_src, size_t(c->Ca));
      for (int s = 0; s < c->Ca; ++s)
        for (size_t k = 0; k < D; ++k) out[D * size_t(src[s]) + k] = x[k * c->Ca + s];
      store(*c, dcams, out.data(), out.size());
    }
    if (dpoints) {
      std::vector<double> d, out(3 * size_t(c->P), 0.0);
      download(*c, d, c->dp, 3 * size_t(c->Pa));
      download(*c, src, c->pt_src, size_t(c->Pa));
      for (int r = 0; r < c->Pa; ++r)
        for (int k = 0; k < 3; ++k)
          out[3 * size_t(c->pt_user[src[r]]) + k] = d[3 * size_t(r) + k];
      store(*c, dpoints, out.data(), out.size());
    }
    return BA_OK;
  });
}

ba_status ba_get_normal_blocks(const ba_ctx* cc, double* U, double* gcv, double* V,
                               double* gpv) {
  ba_ctx* c = const_cast<ba_ctx*>(cc);
  return guarded(c, [&]() -> ba_status {
    if (!c->blocks_valid) return fail(c, BA_ERR_STATE, "no linearisation is available");
    std::vector<int> csrc, psrc;
    download(*c, csrc, c->cam_src, size_t(c->Ca));
    download(*c, psrc, c->pt_src, size_t(c->Pa));
    if (U || gcv) {
      const int D = c->D;
      const size_t ns = size_t(D) * (D + 1) / 2;
      std::vector<double> u, g, Uo(size_t(D) * D * size_t(c->C), 0.0), go(size_t(D) * c->C, 0.0);
      download(*c, u, c->Uraw, ns * size_t(c->Ca));
      download(*c, g, c->gc, size_t(D) * c->Ca);
      for (int s = 0; s < c->Ca; ++s) {
        const size_t cam = size_t(csrc[s]);
        for (int i = 0; i < D; ++i) {
          go[D * cam + i] = g[size_t(i) * c->Ca + s];
          for (int j = 0; j < D; ++j) {
            const int a = std::min(i, j), b = std::max(i, j);
            const int idx = a * D - (a * (a - 1)) / 2 + (b - a);
            Uo[size_t(D) * D * cam + D * i + j] = u[ns * size_t(s) + idx];
          }
        }
      }
      if (U) store(*c, U, Uo.data(), Uo.size());
      if (gcv) store(*c, gcv, go.data(), go.size());
    }
    if (V || gpv) {
      std::vector<double> Vo(9 * size_t(c->P), 0.0), go(3 * size_t(c->P), 0.0), g, v;
      download(*c, g, c->gp, 3 * size_t(c->Pa));
      download(*c, v, static_cast<const double*>(c->V), 6 * size_t(c->Pa));
      static const int m3[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
      for (int r = 0; r < c->Pa; ++r) {
        const size_t pu = size_t(c->pt_user[psrc[r]]);
        for (int i = 0; i < 3; ++i) {
          go[3 * pu + i] = g[3 * size_t(r) + i];
          for (int j = 0; j < 3; ++j) Vo[9 * pu + 3 * i + j] = v[6 * size_t(r) + m3[i][j]];
        }
      }
      if (V) store(*c, V, Vo.data(), Vo.size());
      if (gpv) store(*c, gpv, go.data(), go.size());
    }
    return BA_OK;
  });
}

ba_status ba_get_preconditioner(const ba_ctx* cc, double* Minv) {
  ba_ctx* c = const_cast<ba_ctx*>(cc);
  return guarded(c, [&]() -> ba_status {
    if (!Minv) return fail(c, BA_ERR_ARG, "Minv is NULL");
    if (!c->blocks_valid) return fail(c, BA_ERR_STATE, "no LM system has been set up");
    const int D = c->D;
    const size_t ns = size_t(D) * (D + 1) / 2;
    std::vector<int> csrc;
    std::vector<double> m, out(size_t(D) * D * size_t(c->C), 0.0);
    download(*c, csrc, c->cam_src, size_t(c->Ca));
    download(*c, m, c->Minv, ns * size_t(c->Ca));
    for (int s = 0; s < c->Ca; ++s) {
      const size_t cam = size_t(csrc[s]);
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
          const int a = std::min(i, j), b = std::max(i, j);
          const int idx = a * D - (a * (a - 1)) / 2 + (b - a);
          out[size_t(D) * D * cam + D * i + j] = m[size_t(idx) * c->Ca + s];
        }
    }
    store(*c, Minv, out.data(), out.size());
    return BA_OK;
  });
}

ba_status ba_adjoint(ba_ctx* c, const double* grad_cams, const double* grad_points,
                     float* grad_xy, float* grad_depth) {
  return guarded(c, [&]() -> ba_status {
    if (!c->have_obs) return fail(c, BA_ERR_STATE, "ba_set_observations has not been called");
    if (!grad_cams || !grad_points || !grad_xy)
      return fail(c, BA_ERR_ARG, "grad_cams, grad_points and grad_xy are required");
    if (c->D != 6)
      return fail(c, BA_ERR_STATE, "the adjoint covers poses and points: refine_focal must be off");
    const bool metric = c->have_priors && c->lam_d > 0;
    if (c->n_fixed < 1 || (!metric && c->n_fixed < 2))
      return fail(c, BA_ERR_STATE,
                  "the adjoint needs a fixed gauge: >= 1 fixed camera and depth rows "
                  "(lambda_d > 0), or >= 2 fixed cameras");
    const bool ok = c->opt.precision == BA_PRECISION_FP64
                        ? adjoint_impl<double>(*c, grad_cams, grad_points, grad_xy, grad_depth)
                        : adjoint_impl<float>(*c, grad_cams, grad_points, grad_xy, grad_depth);
    return ok ? BA_OK : BA_NOT_CONVERGED;
  });
}

ba_status ba_kernel_stats(const ba_ctx* cc, ba_kernel_stat* out, int32_t max, int32_t* n) {
  ba_ctx* c = const_cast<ba_ctx*>(cc);
  return guarded(c, [&]() -> ba_status {
    if (!n || (max > 0 && !out)) return fail(c, BA_ERR_ARG, "NULL output");
    int k = 0;
    for (const KStat& s : c->stats) {
      if (k >= max) break;
      std::memset(&out[k], 0, sizeof(ba_kernel_stat));
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", s.name.c_str());
      out[k].launches = s.launches;
      out[k].total_ms = s.ms;
      out[k].total_bytes = s.bytes;
      ++k;
    }
    *n = k;
    return BA_OK;
  });
}

ba_status ba_reset_kernel_stats(ba_ctx* c) {
  return guarded(c, [&]() -> ba_status {
    for (KStat& s : c->stats) {
      s.launches = 0;
      s.ms = 0;
      s.bytes = 0;
    }
    return BA_OK;
  });
}

int64_t ba_device_bytes(const ba_ctx* c) {
  return c ? c->par.bytes + c->obs.bytes + c->ex.bytes + c->ex_bytes : 0;
}

const char* ba_last_error(const ba_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

void ba_destroy(ba_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  delete c;
}

}  // extern "C"
