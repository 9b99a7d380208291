// Internal interface between the host orchestration (ba_api.hip) and the gfx950 kernels
// (ba_kernels.hip). Not installed; the public ABI is include/ba.h.
//
// Layout conventions
//   * compact camera slots: [0, Ca) are the active cameras in ascending original index
//     (Eq. (15) ranks), [Ca, Ca + Cf) the fixed cameras; observations carry their slot.
//   * per-camera solve vectors (x, r, u, p, s, w, b, gc) and blocks (Minv, Ustar) are stored
//     structure-of-arrays: element i of camera s lives at [i * Ca + s].
//   * the camera-major pass reads one aligned 4-vector per observation: the camera-frame
//     point at the linearisation point and the robust weight.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace iba {

constexpr int kBlock = 256;           // threads per block for streaming kernels

// Camera table entry: rotation (row-major, world to camera), centre, intrinsics.
template <typename T>
struct Cam {
  T R[9];
  T c[3];
  T f, cx, cy;
};

// Aligned 4-vector (one 16-byte load in float, two in double).
template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T x, y, z, w;
};

// Packed 3-vector (no padding): the per-observation z of the PCG passes.
template <typename T>
struct P3 {
  T x, y, z;
};

// Per-slot record read by the PCG point pass: rotation, centre and focal length (the values
// of the T camera table, so that X_c = R (X - c) formed from it equals the other kernels'),
// and the current camera direction u of the Schur matvec; 20 values. The float64 pass reads
// X_c from its stream, so its record has no centre (16 values, one 128-byte line).
template <typename T>
struct alignas(4 * sizeof(T)) MvCam {
  T R[9];
  T c[3];
  T f;
  T u[6];
  T pad;
};
template <>
struct alignas(128) MvCam<double> {
  double R[9];
  double f;
  double u[6];
};
// With the focal length refined the camera unknown has a seventh component.
template <typename T>
struct alignas(4 * sizeof(T)) MvCamF {
  T R[9];
  T c[3];
  T f;
  T u[7];
};
template <>
struct alignas(32) MvCamF<double> {
  double R[9];
  double f;
  double u[7];
  double pad[3];
};
template <typename T, int D>
struct MvRecOf {
  using type = MvCam<T>;
};
template <typename T>
struct MvRecOf<T, 7> {
  using type = MvCamF<T>;
};
// Global positioning: the camera unknown is its centre (3 values); the point pass only needs u.
template <typename T>
struct alignas(4 * sizeof(T)) GpMv {
  T u[3];
  T pad;
};
template <typename T>
struct MvRecOf<T, 3> {
  using type = GpMv<T>;
};
template <typename T, int D>
using MvRec = typename MvRecOf<T, D>::type;
// the point pass stages the records in LDS as 16-byte chunks
static_assert(sizeof(MvCam<float>) == 80 && sizeof(MvCamF<float>) == 80, "record layout");
static_assert(sizeof(MvCam<double>) == 128 && sizeof(MvCamF<double>) == 160, "record layout");

// Entries of a symmetric D x D block stored as its upper triangle.
constexpr int sym_count(int D) { return D * (D + 1) / 2; }

// Residual-model constants shared by the kernels.
struct Model {
  double lam_d;       // weight of the inverse-depth row (0: no depth row)
  double huber;       // Huber threshold on the stacked norm (<= 0: plain L2)
  double min_depth;   // validity: z > min_depth
  double filter_px;   // validity: 2-D error <= filter_px (<= 0: off)
  int img_w, img_h;   // validity: projection inside [0, w) x [0, h)
};

// Device-side PCG scalars (one instance per context). The iteration is the
// Chronopoulos-Gear form of preconditioned CG: one fused reduction per iteration.
// Iteration k reads gamma and alpha of iteration k-1 from slot (k+1)&1 and writes its own to
// slot k&1, so the workgroups of one update never read a value written in the same launch.
// The host bounds the iteration count; done is set only on convergence or breakdown, which
// every workgroup of the update decides identically.
struct PcgState {
  double gam[2];      // r.u (u = M^-1 r) by iteration parity
  double alp[2];      // step length by iteration parity
  double bb;          // b.b
  double rr;          // r.r at the last convergence check
  double tol2;        // (relative tolerance)^2
  int iter;           // solution updates so far
  int matvecs;        // Schur matvecs whose result was used
  int max_iter;
  int done;
  int breakdown;      // non-positive curvature or non-finite scalar
  int pad;
};

// Per-launch timing: the next kernel launched by this host thread records its start and
// end in these events (both created by the caller; nullptr disarms).
void set_launch_events(hipEvent_t start, hipEvent_t stop);
// Number of kernel launches issued by this host thread so far.
int64_t launches_issued();

// Compact problem view shared by the point-major and camera-major passes.
template <typename T>
struct Compact {
  int Pa, Ca, Cf;         // active points, active cameras, fixed cameras
  const int* off;         // Pa + 1: point-major CSR over compact observations
  const int* cam;         // Nh: compact camera slot of each observation
  const float2* xy;       // Nh
  const float* depth;     // Nh: prior depth, 0 where invalid (m = 0)
  const int* cam_src;     // Ca + Cf: original camera index of each slot
  const int* cm_off;      // Ca + 1: camera-major segments
  const int* cm_pt;       // Nc: point rank of each camera-major observation
  const int* pm_cm;       // Nh: camera-major position of each observation (solve slots only)
  const double* Xd;       // Pa x 3 compact points (float64)
  const T* Xt;            // Pa x 3 compact points (T)
  const Cam<double>* camd;// Ca + Cf compact camera table (float64)
  const Cam<T>* camt;     // Ca + Cf compact camera table (T)
};

// Per-observation metric data written by the linearisation. The LM step weighs an
// observation by M = w I (w = rho'). The adjoint uses the robust-corrected metric
// M = rho' I + 2 rho'' e e^T; for the Huber function in its linear regime this equals
// w (I - eh eh^T) with eh = e / |e|, so the adjoint stores eh (zero in the quadratic regime)
// and every kernel projects the rows of de/dX_c with (I - eh eh^T).
template <typename T>
struct ObsMetric {
  T* w;          // Nh: rho'
  T* eh;         // Nh x 3: unit residual direction (adjoint only, else nullptr)
  V4<T>* pm_xcw; // Nh: camera-frame point and w, point-major order (float64, and the
                 //     explicit solver; else nullptr: the float32 point pass forms X_c)
  V4<T>* xcw;    // Nc: camera-frame point and w, camera-major order
  V4<T>* cm_e;   // Nc: residual e (3, w slot unused) at the linearisation point, camera-major
  T* cm_eh;      // Nc x 3 (adjoint only)
  T* ce;         // Nh x 3: c = rho' e (adjoint with the full Hessian only, else nullptr): the
                 //     second-order residual and retraction terms of the exact Hessian
  T* cm_ce;      // Nc x 3: the same, camera-major
};

// Point data the camera assembly gathers once per observation, packed in one record.
template <typename T>
struct alignas(16) PtRec {
  double hp[3];   // Vinv rhs_p
  T vinv[6];      // damped inverse point block (symmetric 3x3)
};

// Device figures the launchers size persistent grids and LDS tables with.
struct DevLimits {
  int n_cu = 0;            // compute units
  int lds_per_block = 0;   // bytes of LDS one workgroup may use
};

// ------------------------------------------------------------------ extraction
void launch_cam_table(hipStream_t s, int C, const double* cams, const double* intr,
                      Cam<double>* camd, Cam<float>* camf);
// Validity rows per observation, point-major (vrow) and camera-major (vrow_cm, through
// inv_cm: point-major position -> position in the full camera-major order).
void launch_validate(hipStream_t s, int64_t N, const Model& m, const int* pm_cam,
                     const int* pm_pt, const float2* xy, const float* depth,
                     const double* pts, const Cam<double>* camd, const int* inv_cm,
                     uint8_t* vrow, uint8_t* vrow_cm);
// The same with the C camera records staged in LDS when they fit (else launch_validate), over
// a grid of per_cu workgroups per CU.
void launch_validate_lds(hipStream_t s, int64_t N, int C, const Model& m, const int* pm_cam,
                         const int* pm_pt, const float2* xy, const float* depth,
                         const double* pts, const Cam<double>* camd, const int* inv_cm,
                         uint8_t* vrow, uint8_t* vrow_cm, const DevLimits& dl, int per_cu);
void launch_cam_rows(hipStream_t s, int C, const int* cm_off, const uint8_t* vrow_cm,
                     const uint8_t* fixed, int need, uint8_t* act_c);
void launch_point_rows_prune(hipStream_t s, int P, const int* pt_off, const int* pm_cam,
                             const uint8_t* act_c, const uint8_t* fixed, int need,
                             const int* inv_cm, uint8_t* vrow, uint8_t* vrow_cm,
                             uint8_t* act_p, int* changed);
// Exclusive scans of 0/1 flags (device-wide single-pass scans from hipCUB, ba_sort.hip); out
// has n + 1 entries (out[n] = total); temp needs scan_temp_bytes(n) bytes, n < 2^31 - 1.
// scan_cm flags camera-major observation m when it is valid and its camera is not fixed.
size_t scan_temp_bytes(int64_t n);
hipError_t launch_scan_u8(hipStream_t s, int64_t n, const uint8_t* flags, int* out, void* temp,
                          size_t temp_bytes);
hipError_t launch_scan_cm(hipStream_t s, int64_t n, const uint8_t* vrow_cm, const int* cm_cam,
                          const uint8_t* fixed, int* out, void* temp, size_t temp_bytes);
void launch_compact_points(hipStream_t s, int P, const uint8_t* act_p, const int* rank_p,
                           const int* pt_off, const int* pos_pm, const double* pts,
                           int* pt_src, int* off_hat, double* Xd, float* Xf);
// Slots: active cameras get their rank, fixed cameras Ca + fixed_rank, others -1.
void launch_compact_cams(hipStream_t s, int C, const uint8_t* act_c, const int* rank_c,
                         const uint8_t* fixed, const int* fixed_rank, const int* cm_off,
                         const int* pos_cm, int* slot_all, int* cam_src, int* cm_off_hat);
void launch_compact_cam_table(hipStream_t s, int n, const int* cam_src,
                              const Cam<double>* camd, const Cam<float>* camf,
                              Cam<double>* camd_hat, Cam<float>* camf_hat);
// Compact point-major observations, and for those of solve cameras (slots < Ca) their
// camera-major position pm_cm and the point rank there (cm_pt); pm_cm = -1 otherwise.
void launch_compact_obs(hipStream_t s, int64_t N, const uint8_t* vrow, const int* pos_pm,
                        const int* pm_cam, const int* slot_all, const float2* pm_xy,
                        const float* pm_depth, const int* pm_orig, int Ca, const int* inv_cm,
                        const int* pos_cm, const int* pm_pt, const int* rank_p, int* cam_hat,
                        float2* xy_hat, float* depth_hat, int* orig_hat, int* pm_cm,
                        int* cm_pt);
// Matvec records of every slot (R, f from the compact table; u = 0).
template <typename T>
void launch_mv_table(hipStream_t s, int D, int n, const Cam<double>* camd_hat, void* mvt);

// ------------------------------------------------------------------ linearisation
// Per point: residuals (float64), robust weights, V = J_p^T M J_p (T products accumulated in
// float64), gp = J_p^T M e (float64); per block: cost, sum |r_2d|^2 and max |gp| into
// partials[3 * block]. Per observation the (X_c, w) stream in both orders, and e (and eh in
// adjoint mode) at the camera-major position of the observations of solve cameras.
// G lanes per point; one workgroup per 256 points, grid lin_point_blocks(Pa) (partials
// needs 3 doubles per workgroup).
inline int lin_point_blocks(int Pa) { return ((Pa + kBlock - 1) / kBlock + 7) / 8 * 8; }
inline int lin_point_blocks_lds(int Pa) { return ((Pa + 1023) / 1024 + 7) / 8 * 8; }
// Returns the number of partial triples written (one per workgroup).
template <typename T>
int launch_lin_point(hipStream_t s, bool adj, int G, const Model& m, const Compact<T>& cp,
                     ObsMetric<T> om, double* V, double* gp, double* partials,
                     const DevLimits& dl);
// V* = V + lam clamp(diag V); Vinv (inverted in float64, stored as T); hp = Vinv rhs_p.
// rhs_p = -gp when rhs_p == nullptr.
template <typename T>
void launch_point_damp(hipStream_t s, int Pa, double lam, double dmin, double dmax,
                       const double* V, const double* gp, const double* rhs_p, T* Vinv,
                       double* hp, PtRec<T>* prec, int* bad);
// Items of the camera pass. A camera's segment of camera-major positions (sorted by point
// rank) is split at the boundaries of R point ranges (R = 1, or 8: the eighths of the point
// ranks that the point pass gives the 8 XCDs), and every piece is cut into items of at most K
// positions. A camera's items are numbered consecutively from off[s] (off[Ca] = the item
// count), so the update kernel sums their partials in a fixed order. at[r * cap + q] describes
// the q-th item of range r as (item, camera, first position, end position), or has item -1
// past the range's last item: the camera pass takes range r's items on the workgroups of XCD
// r, whose L2 holds that range's point vectors z after the point pass, and reads one record
// per item. Built on the device by the PCG init.
constexpr int kMaxRanges = 8;
struct CamItems {
  int R, cap;   // ranges; capacity of each range's list in at
  int* off;     // Ca + 2: off[Ca + 1] = the largest item count of a range
  int4* at;     // R * cap
  int slots;    // slots per range the camera pass covers (<= cap; set from off[Ca + 1])
};
// Item size: K = Nc / kCamChunks rounded up to a multiple of 64, at least 512, so that
// nchunks = ceil(Nc / K) <= kCamChunks. There are at most R Ca + nchunks items in all (each
// camera's piece of a range adds one partial item at most) and at most Ca + nchunks in a range.
constexpr int kCamChunks = 1024;
inline void cam_chunking(int Nc, int& K, int& nchunks) {
  const int per = (Nc + kCamChunks - 1) / kCamChunks;
  K = per <= 512 ? 512 : (per + 63) / 64 * 64;
  nchunks = Nc > 0 ? (Nc + K - 1) / K : 0;
}
// rb[r * Ca + s] = the first position of camera s's segment whose point rank is at least
// r * ppx (r = 1 .. R - 1; row 0 is the segment start).
void launch_range_bounds(hipStream_t s, int Ca, int R, int ppx, const int* cm_off,
                         const int* cm_pt, int* rb);
// Builds the items: K positions at most, R ranges cut at rb (R = 1: rb unused).
void launch_build_items(hipStream_t s, int Ca, const int* cm_off, const int* rb, int K,
                        CamItems it);
// Camera assembly. launch_cam_items: per item of `it` (positions in one point range, so the
// gathered point records stay in one XCD's L2) the rows sum W Vinv W^T (D (D + 1) / 2) and
// sum W hp (D) (schur), or U = J_c^T M J_c (D (D + 1) / 2) and g_c (D) (!schur), into
// part[item * 2 (D (D + 1) / 2 + D) + row] (see part_rows); nslot is the item capacity.
// launch_cam_assemble: per camera slot its items' rows (item_off) added in item order, then
// b = rhs_c - sum W hp, S_cc = U* - sum W Vinv W^T and its inverse (Cholesky, float64).
// rhs_c = -gc when rhs_c == nullptr. SoA outputs. Scc (optional, SoA like Minv) receives S_cc
// itself for the explicit reduced system.
template <typename T>
void launch_cam_items(hipStream_t s, bool adj, bool schur, int D, const Model& m,
                      const Compact<T>& cp, ObsMetric<T> om, const PtRec<T>* prec, CamItems it,
                      int nslot, double* part, const DevLimits& dl);
template <typename T>
void launch_cam_assemble(hipStream_t s, int D, int Ca, double lam, double dmin, double dmax,
                         const int* item_off, const double* part, const double* rhs_c,
                         double* Uraw, T* Ustar, double* gc, double* b, double* Minv,
                         double* Scc = nullptr);

// ------------------------------------------------------------------ PCG on S
// x = 0, r = b, u = M^-1 r (also into the matvec records), p = s = 0, Uu = U* u and the
// per-camera terms r.u, u.U*u, r.r of iteration 0 (terms: 2 x 3 arrays of Ca, SoA, the
// first three for even iterations); the camera-pass items: camera s owns items
// item_off[s] .. item_off[s + 1] - 1 (item_cam[i] = s), one per K positions of its segment.
template <typename T>
void launch_pcg_init(hipStream_t s, int D, int Ca, const double* b, const double* Minv,
                     const T* Ustar, double* x, double* r, double* u, double* p, double* sv,
                     double* Uu, double* terms, void* mvt, PcgState* st, double tol2,
                     int max_iter);
// Camera-side launchers take the camera dimension D: 6 (pose) or 7 (pose and focal length,
// matvec records MvCamF); the adjoint mode runs with D = 6 only.

// z_p = Vinv sum_k W_k^T u_c (point-major pass, G lanes per point), one 3-vector per point
// rank (zq, Pa entries). When the Ca matvec records fit in LDS, a persistent grid stages them
// there, XCD x taking the x-th eighth of the point ranks.
template <typename T>
void launch_schur_point(hipStream_t s, bool adj, int D, int G, const Model& m,
                        const Compact<T>& cp, ObsMetric<T> om, const void* mvt, const T* Vinv,
                        P3<T>* zq, const PcgState* st, const DevLimits& dl);
// Camera-major pass over the items: per item i, sum_k W_k z_k over its positions, z gathered
// through the position's point rank (part: rows 0..D-1 of nslot entries, SoA) and that sum's
// dot with u_s (row D). nslot >= the item count; one workgroup per slot, R it.slots.
template <typename T>
void launch_schur_cam(hipStream_t s, bool adj, int D, const Model& m, const Compact<T>& cp,
                      ObsMetric<T> om, const double* u, const P3<T>* zq, CamItems it,
                      int nslot, double* part, const PcgState* st, const DevLimits& dl);
// w = U* u - (each camera's item partials; nit items in all), fused reduction of the per-camera
// terms, convergence
// test, then p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = M^-1 r, and U* u
// with the next iteration's terms.
template <typename T>
void launch_pcg_update(hipStream_t s, int D, int Ca, int k, const double* Minv, const T* Ustar,
                       const int* item_off, int nit, int nslot, const double* part,
                       double* terms, double* x, double* r, double* u, double* p, double* sv,
                       double* Uu, void* mvt, PcgState* st);
// The true residual of a PCG solution x: k_x_to_mv writes x into the matvec records and
// clears the done flag of st (a state used only for this product), the two matvec passes run
// with st, and launch_true_residual forms |b - S x|^2 and |b|^2 into out[0], out[1].
template <typename T>
void launch_x_to_mv(hipStream_t s, int D, int Ca, const double* x, void* mvt, PcgState* st);
template <typename T>
void launch_true_residual(hipStream_t s, int D, int Ca, const double* x, const double* b,
                          const T* Ustar, const int* item_off, int nslot, const double* part,
                          double* out);
// Back-substitution dp = Vinv (b_p - sum_k W_k^T x_c) = hp - z per point: hp = Vinv b_p from
// launch_point_damp, z = Vinv sum_k W_k^T x_c from launch_schur_point run on the matvec records
// holding x (launch_x_to_mv); use_z = false (no solve camera) gives dp = hp.
template <typename T>
void launch_backsub(hipStream_t s, int Pa, const double* hp, const P3<T>* zq, bool use_z,
                    double* dp);

// ------------------------------------------------------------------ candidate
// Candidate camera table over all slots (retracted for s < Ca, copied for fixed slots).
// (D = 7: the focal length of the candidate is f + x_f)
void launch_cam_candidate(hipStream_t s, int Ca, int Cf, int D, const int* cam_src,
                          const double* x, const double* cams, const Cam<double>* camd_hat,
                          double* cand_cams, Cam<double>* cand_tab);
// Candidate cost terms over lin_point_blocks* workgroups (5 partials per workgroup; returns the
// workgroup count).
template <typename T>
int launch_point_candidate(hipStream_t s, const Model& m, const Compact<T>& cp, int D,
                           const Cam<double>* cand_tab, const double* x, const double* dp,
                           const double* gp, const T* w, double* Xcand, double* partials,
                           const DevLimits& dl);
// Sums per-block partials (K doubles per block) in a fixed order; with gc != nullptr also
// out[K] = gc . x over the ncu camera unknowns and out[K + 1] = max |gc|.
void launch_reduce_partials(hipStream_t s, int nblocks, int K, const double* partials,
                            unsigned max_mask, int ncu, const double* gc, const double* x,
                            double* out);
// Accepted candidate into the full arrays; intr != nullptr also takes the refined focal.
void launch_scatter(hipStream_t s, int Pa, int Ca, const int* pt_src, const double* Xcand,
                    const int* cam_src, const double* cand_cams, const Cam<double>* cand_tab,
                    double* pts, double* cams, double* intr);

// ------------------------------------------------------------------ adjoint
// rhs for the adjoint solve: tangent-mapped camera gradients (SoA) and point gradients, both
// gathered from caller-order device arrays.
void launch_adjoint_rhs(hipStream_t s, int Ca, int Pa, const int* cam_src, const double* cams,
                        const double* grad_cams, const int* pt_src, const int* pt_user,
                        const double* grad_pts, double* rhs_c, double* rhs_p);
template <typename T>
void launch_adjoint_obs(hipStream_t s, const Model& m, const Compact<T>& cp, ObsMetric<T> om,
                        const double* x, const double* dp, const int* orig, float* gxy,
                        float* gdepth);

// ------------------------------------------------------------------ explicit reduced system
// The reduced camera system S = U* - W V*^-1 W^T assembled as D x D blocks (a solver variant of
// the matrix-free Schur PCG). Off-diagonal block (i, j) = - sum over the points p seen by both
// cameras of W_ip V*_p^-1 W_jp^T; the diagonal blocks S_cc come from the camera assembly.
//
// hipCUB primitives (ba_sort.hip): stable radix sort of 32-bit keys with 64-bit values over
// the low end_bit bits of the keys, exclusive prefix sum of int64.
size_t sort_pairs64_temp_bytes(int n, int end_bit);
hipError_t sort_pairs64(void* temp, size_t temp_bytes, const uint32_t* keys_in,
                        uint32_t* keys_out, const uint64_t* vals_in, uint64_t* vals_out, int n,
                        int end_bit, hipStream_t s);
size_t exclusive_sum_temp_bytes(int n);
hipError_t exclusive_sum(void* temp, size_t temp_bytes, const int64_t* in, int64_t* out, int n,
                         hipStream_t s);
// Per active point: cnt[r] = m (m - 1) with m its observations in solve cameras (ordered pairs
// of distinct observations), and the point rank of every point-major observation.
template <typename T>
void launch_pair_counts(hipStream_t s, const Compact<T>& cp, int64_t* cnt, int* pm_rank);
// Contribution c = coff[r] + (pairs of point r in order): key = cam(a) Ca + cam(b), value =
// the point-major positions of a (high 32 bits) and b (low 32 bits).
template <typename T>
void launch_pair_keys(hipStream_t s, const Compact<T>& cp, const int64_t* coff, uint32_t* key,
                      uint64_t* val);
// Flags of run starts in the sorted keys (1 where key differs from its predecessor).
void launch_run_flags(hipStream_t s, int64_t n, const uint32_t* key, int64_t* flag);
// Block list from the run starts: bkey[b], bstart[b] (the first sorted position of block b).
void launch_block_list(hipStream_t s, int64_t n, const uint32_t* key, const int64_t* flag,
                       const int64_t* bidx, uint32_t* bkey, int64_t* bstart);
// Row pointers of the block rows (blocks are sorted row-major): row_ptr[i] = first block of
// row >= i, i = 0..Ca.
void launch_block_rows(hipStream_t s, int Ca, int64_t nb, const uint32_t* bkey, int64_t* row_ptr);
// One wave per off-diagonal block: S_b = - sum over its contributions (sorted order) of
// W_k V*^-1 W_l^T, stored row-major D x D in T.
template <typename T>
void launch_schur_blocks(hipStream_t s, int D, const Model& m, const Compact<T>& cp,
                         ObsMetric<T> om, const T* Vinv, const int* pm_rank, int64_t nb,
                         const uint32_t* bkey, const int64_t* bstart, const uint64_t* sval,
                         T* sblk);
// One wave per block row: w_i = S_cc u_i + sum_b S_b u_col(b), written as the single item
// partial Uu_i - w_i (and its dot with u_i) that the PCG update consumes.
template <typename T>
void launch_schur_spmv(hipStream_t s, int D, int Ca, const int64_t* row_ptr,
                       const uint32_t* bkey, const T* sblk, const double* Scc, const double* u,
                       const double* Uu, int nslot, double* part, const PcgState* st);

// ------------------------------------------------------------------ global positioning
// Depth-constrained global positioning (Eqs. (1), (4), (5), (8)): rotations fixed, unknowns the
// camera centres (3 per camera, PCG with D = 3), the points and the free per-observation scales
// (eliminated per observation before the points). Residual u = v - s (X - c) on the unit world
// ray v = R^T a / |a|, a = K^-1 [x, y, 1]; a valid depth prior pins s = 1 / (d_hat |a|).
//
// Per compact observation the linearisation keeps, in both orders: d = X - c, the scale (stored
// negated when pinned), u and the robust weight w.
template <typename T>
struct alignas(8 * sizeof(T)) GpLin {
  T d[3];
  T s;
  T u[3];
  T w;
};
// After eliminating a free scale with its damped diagonal h* = h + lambda clamp(h), h = w |d|^2,
// the observation couples its camera centre and point through A = a0 I - e e^T with
// a0 = w s^2 and e = (w s / sqrt(h*)) d (e = 0 when pinned); the record stores (e, a0).

// Row counts (3 pinned, 2 free, 0 with non-finite data) in both orders.
void launch_gp_validate(hipStream_t s, int64_t N, const float2* pm_xy, const float* pm_depth,
                        const int* inv_cm, uint8_t* vrow, uint8_t* vrow_cm);
// Free scales (user order) at the inverse distance of the current estimate; pinned ones at
// 1 / (d_hat |a|).
void launch_gp_init_scales(hipStream_t s, int64_t N, const int* pm_cam, const int* pm_pt,
                           const int* pm_orig, const float2* pm_xy, const float* pm_depth,
                           const double* pts, const Cam<double>* camd, double* scales);
// Residuals, weights, the records above, g_X = -sum w s u per point (gX, P x 3) and block
// partials {cost, sum |u|^2, max |g|} (3 per block of lin_point_blocks(Pa)).
template <typename T>
int launch_gp_lin(hipStream_t s, int G, const Compact<T>& cp, const int* orig,
                  const double* scales, double delta, GpLin<T>* lin_pm, GpLin<T>* lin_cm,
                  double* gX, double* partials, const DevLimits& dl);   // returns the partials
// Per point: the (e, a0) records in both orders, V* = sum A + lambda clamp(sum a0) I inverted
// in float64, hp = V*^-1 r_X with r_X = sum w s (u + d g_s / h*), packed into prec.
template <typename T>
void launch_gp_point_setup(hipStream_t s, int G, const Compact<T>& cp, double lam, double dmin,
                           double dmax, const GpLin<T>* lin_pm, V4<T>* a_pm, V4<T>* a_cm,
                           T* Vinv, double* hp, PtRec<T>* prec, int* bad);
// Per camera: U* = sum A + lambda clamp(sum a0) I, g_c = sum w s u, b = r_c + sum A hp with
// r_c = -sum w s (u + d g_s / h*), S_cc = U* - sum A V*^-1 A and its inverse (SoA, D = 3).
template <typename T>
void launch_gp_cam_assemble(hipStream_t s, const Compact<T>& cp, double lam, double dmin,
                            double dmax, const GpLin<T>* lin_cm, const V4<T>* a_cm,
                            const PtRec<T>* prec, T* Ustar, double* gc, double* b,
                            double* Minv);
// The two PCG passes of S u = U* u - sum_c A V*^-1 sum_p A u (camera records GpMv).
template <typename T>
void launch_gp_schur_point(hipStream_t s, int G, const Compact<T>& cp, const V4<T>* a_pm,
                           const void* mvt, const T* Vinv, P3<T>* zq_cm, const PcgState* st,
                           const DevLimits& dl);
template <typename T>
void launch_gp_schur_cam(hipStream_t s, const Compact<T>& cp, const V4<T>* a_cm,
                         const double* u, const P3<T>* zq_cm, CamItems it, int nslot,
                         double* part, const PcgState* st, const DevLimits& dl);
// dX = hp + V*^-1 sum A dc.
template <typename T>
void launch_gp_backsub(hipStream_t s, int G, const Compact<T>& cp, const V4<T>* a_pm,
                       const T* Vinv, const double* hp, const double* x, double* dp);
// Candidate (float64, recomputed from the compact data): centres c + dc, points X + dX, free
// scales s + ds with ds = (-g_s + w s d.(dc - dX)) / h*; per block {actual decrease, sum w
// |J delta|^2, g_X.dX + g_s ds, scales <= 0, candidate cost} (5 per workgroup of kBlock
// threads, G lanes per point). Returns the number of workgroups.
template <typename T>
int launch_gp_candidate(hipStream_t s, int G, const Compact<T>& cp, const int* orig,
                        const double* scales, double delta, double lam, double dmin,
                        double dmax, const double* x, const double* dp, const double* gX,
                        double* Xcand, double* s_cand, double* partials,
                        const DevLimits& dl);   // returns the number of partials
// Accepted step: points, camera centres (cams C x 7, entries 4..6) and free scales.
void launch_gp_scatter(hipStream_t s, int Pa, int Ca, int64_t Nh, const int* pt_src,
                       const double* Xcand, const int* cam_src, const double* x,
                       const float* depth_hat, const int* orig, const double* s_cand,
                       double* pts, double* cams, double* scales);

}  // namespace iba
