// gfx950 kernels of the LM bundle-adjustment step (InstantSfM, arXiv 2510.13310).
//
// Every kernel streams structure-of-arrays observation data in one of two fixed orders:
//   point-major  (compact observations grouped by point, CSR offsets `off`), one thread per
//                point walks its segment and reduces in registers;
//   camera-major (the same observations grouped by camera, `cm_off`), one block per camera
//                reduces its segment with wave shuffles and LDS in a fixed order.
// No global atomics are used for sums, so every result is bitwise reproducible.
//
// The per-observation Jacobian blocks are never stored: both PCG passes recompute
// de/dX_c, J_c = de/dX_c [I | -[X_c]x] and J_p = de/dX_c R from the point, the camera table
// (a few KB, cache resident) and the stored robust weight. This trades ~60 flops per
// observation for the 72-144 bytes a stored W_k = J_c^T J_p block would cost per pass.
#include "ba_kernels.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace iba {
namespace {

constexpr int kWave = 64;

// ------------------------------------------------------------------ launches
// Events armed by set_launch_events are handed to the next launch on this host thread, which
// records its start and end in them (hipExtLaunchKernel): no extra packets in the stream.
thread_local hipEvent_t g_ev_start = nullptr;
thread_local hipEvent_t g_ev_stop = nullptr;
thread_local int64_t g_launches = 0;

template <typename... KArgs, typename... Args>
void launch_k(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t s,
              Args... args) {
  ++g_launches;
  if (g_ev_start != nullptr) {
    hipEvent_t a = g_ev_start, b = g_ev_stop;
    g_ev_start = g_ev_stop = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, a, b, 0u, static_cast<KArgs>(args)...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, static_cast<KArgs>(args)...);
  }
}

// ------------------------------------------------------------------ reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, kWave);
    v = u > v ? u : v;
  }
  return v;
}

// Sum over aligned groups of G lanes (G = 1, 2, 4, 8 or 16), every lane of a group getting the
// group's sum. float32 uses DPP lane moves within rows of 16 lanes (no trip through the LDS
// crossbar): xor 1 and xor 2 by quad permutations, then the mirror within each 8 lanes and
// within each 16 lanes; after the quad steps all lanes of a quad hold the quad's sum, so a
// mirror pairs each lane with the other half. Every lane adds the same two operands (in
// swapped order), so all lanes of a group hold the bitwise same sum. float64 uses shuffles.
template <int Ctrl>
__device__ __forceinline__ float dpp_move(float x) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), Ctrl, 0xF, 0xF, false));
}
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  static_assert(G >= 1 && G <= 16 && (G & (G - 1)) == 0, "lane groups of 1 to 16");
  if constexpr (G >= 2) v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp_move<0x141>(v);   // row_half_mirror
  if constexpr (G >= 16) v += dpp_move<0x140>(v);  // row_mirror
  return v;
}
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sums K per-thread values over the block; the result is valid in thread 0.
// smem holds K * (blockDim.x / 64) values.
template <typename T, int K>
__device__ __forceinline__ void block_sum(T (&v)[K], T* smem) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) smem[wid * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < K; ++k) {
      T a = smem[k];
      for (int w = 1; w < nw; ++w) a += smem[w * K + k];
      v[k] = a;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ small linear algebra
// Symmetric D x D stored as the upper triangle, row-major (D (D + 1) / 2 values).
template <int D>
__host__ __device__ constexpr int symd(int i, int j) {
  return i <= j ? i * D - (i * (i - 1)) / 2 + (j - i) : j * D - (j * (j - 1)) / 2 + (i - j);
}
__host__ __device__ constexpr int sym6(int i, int j) { return symd<6>(i, j); }
// Symmetric 3x3: [00, 01, 02, 11, 12, 22].
__host__ __device__ constexpr int sym3(int i, int j) {
  return i <= j ? i * 3 - (i * (i - 1)) / 2 + (j - i) : j * 3 - (j * (j - 1)) / 2 + (i - j);
}

template <typename T>
__device__ __forceinline__ void cross3(const T a[3], const T b[3], T o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Camera-frame coordinates R (X - c).
template <typename T, typename S>
__device__ __forceinline__ void cam_frame(const Cam<S>& cm, T X0, T X1, T X2, T Xc[3]) {
  const T d0 = X0 - T(cm.c[0]), d1 = X1 - T(cm.c[1]), d2 = X2 - T(cm.c[2]);
  Xc[0] = T(cm.R[0]) * d0 + T(cm.R[1]) * d1 + T(cm.R[2]) * d2;
  Xc[1] = T(cm.R[3]) * d0 + T(cm.R[4]) * d1 + T(cm.R[5]) * d2;
  Xc[2] = T(cm.R[6]) * d0 + T(cm.R[7]) * d1 + T(cm.R[8]) * d2;
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// R (X - c) in T from T-valued rotation, centre and point, with one fixed order of fused
// multiply-adds: the Jacobian kernels of the solve (streams written by the linearisation,
// the PCG point pass, back-substitution) all form X_c with it, so they see the same bits.
template <typename T>
__device__ __forceinline__ void frame_t(const T R[9], const T c[3], T X0, T X1, T X2,
                                        T Xc[3]) {
  const T d0 = X0 - c[0], d1 = X1 - c[1], d2 = X2 - c[2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    Xc[i] = fma_t(R[3 * i + 2], d2, fma_t(R[3 * i + 1], d1, R[3 * i] * d0));
}

// R v and R^T v for a row-major camera rotation.
template <typename T, typename S>
__device__ __forceinline__ void rot_mul(const Cam<S>& cm, const T v[3], T o[3]) {
  o[0] = T(cm.R[0]) * v[0] + T(cm.R[1]) * v[1] + T(cm.R[2]) * v[2];
  o[1] = T(cm.R[3]) * v[0] + T(cm.R[4]) * v[1] + T(cm.R[5]) * v[2];
  o[2] = T(cm.R[6]) * v[0] + T(cm.R[7]) * v[1] + T(cm.R[8]) * v[2];
}
template <typename T, typename S>
__device__ __forceinline__ void rot_tmul(const Cam<S>& cm, const T v[3], T o[3]) {
  o[0] = T(cm.R[0]) * v[0] + T(cm.R[3]) * v[1] + T(cm.R[6]) * v[2];
  o[1] = T(cm.R[1]) * v[0] + T(cm.R[4]) * v[1] + T(cm.R[7]) * v[2];
  o[2] = T(cm.R[2]) * v[0] + T(cm.R[5]) * v[1] + T(cm.R[8]) * v[2];
}

// 1 / z of a camera-frame depth (z > 0.1 wherever a Jacobian is formed): float32 takes the
// hardware reciprocal (within 1 ulp) instead of the correctly rounded division sequence;
// every float32 Jacobian row goes through AMat or Curv, so all float32 kernels use the same
// value. float64 divides.
__device__ __forceinline__ float recip(float z) { return __builtin_amdgcn_rcpf(z); }
__device__ __forceinline__ double recip(double z) { return 1.0 / z; }

// Rows of de/dX_c (3 x 3): pinhole rows (f/z)[1 0 -x/z], (f/z)[0 1 -y/z] and the
// inverse-depth row [0 0 -lam_d/z^2]. The plain form keeps the five structural non-zeros;
// the projected form (adjoint metric) is a full matrix (I - eh eh^T) A.
template <typename T, bool PROJ>
struct AMat;

template <typename T>
struct AMat<T, false> {
  T a00, a02, a11, a12, a22;
  __device__ __forceinline__ void set(T f, T lam_d, const T Xc[3]) {
    const T iz = recip(Xc[2]);
    a00 = f * iz;
    a11 = a00;
    a02 = -a00 * Xc[0] * iz;
    a12 = -a00 * Xc[1] * iz;
    a22 = -lam_d * iz * iz;
  }
  __device__ __forceinline__ void project(const T*) {}
  __device__ __forceinline__ void apply(const T d[3], T t[3]) const {
    t[0] = a00 * d[0] + a02 * d[2];
    t[1] = a11 * d[1] + a12 * d[2];
    t[2] = a22 * d[2];
  }
  __device__ __forceinline__ void applyT(const T t[3], T m[3]) const {
    m[0] = a00 * t[0];
    m[1] = a11 * t[1];
    m[2] = a02 * t[0] + a12 * t[1] + a22 * t[2];
  }
  __device__ __forceinline__ void row(int i, T r[3]) const {
    r[0] = i == 0 ? a00 : T(0);
    r[1] = i == 1 ? a11 : T(0);
    r[2] = i == 0 ? a02 : (i == 1 ? a12 : a22);
  }
};

template <typename T>
struct AMat<T, true> {
  T a[9];
  __device__ __forceinline__ void set(T f, T lam_d, const T Xc[3]) {
    const T iz = recip(Xc[2]);
    const T fz = f * iz;
    a[0] = fz; a[1] = T(0); a[2] = -fz * Xc[0] * iz;
    a[3] = T(0); a[4] = fz; a[5] = -fz * Xc[1] * iz;
    a[6] = T(0); a[7] = T(0); a[8] = -lam_d * iz * iz;
  }
  // A <- (I - eh eh^T) A, column by column.
  __device__ __forceinline__ void project(const T* eh) {
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const T s = eh[0] * a[l] + eh[1] * a[3 + l] + eh[2] * a[6 + l];
      a[l] -= eh[0] * s;
      a[3 + l] -= eh[1] * s;
      a[6 + l] -= eh[2] * s;
    }
  }
  __device__ __forceinline__ void apply(const T d[3], T t[3]) const {
    t[0] = a[0] * d[0] + a[1] * d[1] + a[2] * d[2];
    t[1] = a[3] * d[0] + a[4] * d[1] + a[5] * d[2];
    t[2] = a[6] * d[0] + a[7] * d[1] + a[8] * d[2];
  }
  __device__ __forceinline__ void applyT(const T t[3], T m[3]) const {
    m[0] = a[0] * t[0] + a[3] * t[1] + a[6] * t[2];
    m[1] = a[1] * t[0] + a[4] * t[1] + a[7] * t[2];
    m[2] = a[2] * t[0] + a[5] * t[1] + a[8] * t[2];
  }
  __device__ __forceinline__ void row(int i, T r[3]) const {
    r[0] = a[3 * i];
    r[1] = a[3 * i + 1];
    r[2] = a[3 * i + 2];
  }
};

// Second-order terms of one observation in the exact Hessian of its cost (the adjoint with
// the full Hessian). With c = rho' e (the observation's cost gradient with respect to its
// residual), a = A^T c is its gradient with respect to X_c (A = de/dX_c, not projected), and
// S = sum_i c_i d^2 e_i / dX_c^2 is the curvature of the pinhole and inverse-depth rows:
//   S02 = -c0 f / z^2, S12 = -c1 f / z^2, S22 = 2 (f (c0 x + c1 y) + lam_d c2) / z^3.
// Together with the second-order part of the left SE(3) retraction of X_c,
// (1/2) [phi]x^2 X_c + [phi]x R dX + (1/2) [phi]x rho, they add to the observation's block:
//   camera-camera  J_c^T S J_c + [[0, [a]x/2], [-[a]x/2, (a X^T + X a^T)/2 - (a.X) I]],
//   camera-point   J_c^T S R + [0 ; -[a]x R],   point-point  R^T S R.
template <typename T>
struct Curv {
  T a[3];
  T s02, s12, s22;
  __device__ __forceinline__ void set(T f, T lam_d, const T Xc[3], const T c[3]) {
    const T iz = recip(Xc[2]);
    const T fz = f * iz;
    const T cxy = c[0] * Xc[0] + c[1] * Xc[1];
    a[0] = fz * c[0];
    a[1] = fz * c[1];
    a[2] = -fz * iz * cxy - lam_d * iz * iz * c[2];
    s02 = -c[0] * fz * iz;
    s12 = -c[1] * fz * iz;
    s22 = T(2) * iz * iz * (fz * cxy + lam_d * c[2] * iz);
  }
  // m += S d
  __device__ __forceinline__ void add_s(const T d[3], T m[3]) const {
    m[0] += s02 * d[2];
    m[1] += s12 * d[2];
    m[2] += s02 * d[0] + s12 * d[1] + s22 * d[2];
  }
};

// Huber on the squared norm s: rho, rho', rho''.
__device__ __forceinline__ void huber(double s, double delta, double& rho, double& d1,
                                      double& d2) {
  if (delta > 0.0 && s > delta * delta) {
    const double rs = sqrt(s);
    rho = 2.0 * delta * rs - delta * delta;
    d1 = delta / rs;
    d2 = -0.5 * delta / (rs * rs * rs);
  } else {
    rho = s;
    d1 = 1.0;
    d2 = 0.0;
  }
}

// Stacked residual e = [Pi - x ; lam_d (1/z - m/d_hat)] of one observation (float64).
__device__ __forceinline__ void residual(const Cam<double>& cm, const double Xc[3], float2 xy,
                                        float depth, double lam_d, double e[3]) {
  const double iz = 1.0 / Xc[2];
  e[0] = cm.f * Xc[0] * iz + cm.cx - double(xy.x);
  e[1] = cm.f * Xc[1] * iz + cm.cy - double(xy.y);
  const double dinv = depth > 0.0f ? 1.0 / double(depth) : 0.0;
  e[2] = lam_d * (iz - dinv);
}

// ------------------------------------------------------------------ extraction kernels
__global__ void __launch_bounds__(kBlock)
k_cam_table(int C, const double* __restrict__ cams, const double* __restrict__ intr,
            Cam<double>* __restrict__ camd, Cam<float>* __restrict__ camf) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double qw = cams[7 * c], qx = cams[7 * c + 1], qy = cams[7 * c + 2], qz = cams[7 * c + 3];
  const double n = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw /= n; qx /= n; qy /= n; qz /= n;
  Cam<double> d;
  d.R[0] = 1 - 2 * (qy * qy + qz * qz);
  d.R[1] = 2 * (qx * qy - qw * qz);
  d.R[2] = 2 * (qx * qz + qw * qy);
  d.R[3] = 2 * (qx * qy + qw * qz);
  d.R[4] = 1 - 2 * (qx * qx + qz * qz);
  d.R[5] = 2 * (qy * qz - qw * qx);
  d.R[6] = 2 * (qx * qz - qw * qy);
  d.R[7] = 2 * (qy * qz + qw * qx);
  d.R[8] = 1 - 2 * (qx * qx + qy * qy);
  d.c[0] = cams[7 * c + 4];
  d.c[1] = cams[7 * c + 5];
  d.c[2] = cams[7 * c + 6];
  d.f = intr[3 * c];
  d.cx = intr[3 * c + 1];
  d.cy = intr[3 * c + 2];
  camd[c] = d;
  Cam<float> f;
  for (int i = 0; i < 9; ++i) f.R[i] = float(d.R[i]);
  for (int i = 0; i < 3; ++i) f.c[i] = float(d.c[i]);
  f.f = float(d.f);
  f.cx = float(d.cx);
  f.cy = float(d.cy);
  camf[c] = f;
}

// Validity of every observation (Eq. (10) + frustum + reprojection filter), written as the
// number of residual rows it contributes (0 when invalid).
__global__ void __launch_bounds__(kBlock)
k_validate(int64_t N, Model m, const int* __restrict__ pm_cam, const int* __restrict__ pm_pt,
           const float2* __restrict__ xy, const float* __restrict__ depth,
           const double* __restrict__ pts, const Cam<double>* __restrict__ camd,
           const int* __restrict__ inv_cm, uint8_t* __restrict__ vrow,
           uint8_t* __restrict__ vrow_cm) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const Cam<double> cm = camd[pm_cam[k]];
  const int p = pm_pt[k];
  double Xc[3];
  cam_frame(cm, pts[3 * p], pts[3 * p + 1], pts[3 * p + 2], Xc);
  bool ok = Xc[2] > m.min_depth;
  if (ok) {
    const double u = cm.f * Xc[0] / Xc[2] + cm.cx;
    const double v = cm.f * Xc[1] / Xc[2] + cm.cy;
    ok = u >= 0.0 && u < double(m.img_w) && v >= 0.0 && v < double(m.img_h);
    if (ok && m.filter_px > 0.0) {
      double e[3];
      residual(cm, Xc, xy[k], 0.0f, 0.0, e);
      ok = e[0] * e[0] + e[1] * e[1] <= m.filter_px * m.filter_px;
    }
  }
  const int rows = 2 + ((m.lam_d > 0.0 && depth[k] > 0.0f) ? 1 : 0);
  const uint8_t v = ok ? uint8_t(rows) : uint8_t(0);
  vrow[k] = v;
  vrow_cm[inv_cm[k]] = v;
}

// Copies n float64 camera records into LDS (all B threads of the workgroup take part) and
// returns the LDS copy.
template <int B>
__device__ __forceinline__ const Cam<double>* stage_cams(const Cam<double>* __restrict__ src,
                                                         int n, double* lds) {
  const int nwords = n * int(sizeof(Cam<double>) / sizeof(double));
  const double* w = reinterpret_cast<const double*>(src);
  for (int i = threadIdx.x; i < nwords; i += B) lds[i] = w[i];
  __syncthreads();
  return reinterpret_cast<const Cam<double>*>(lds);
}

// The same over a grid-stride walk with the camera table staged in LDS (C records of 120 B),
// so the per-observation camera reads hit LDS instead of L2.
constexpr int kLdsWalkBlock = 1024;

__global__ void __launch_bounds__(kLdsWalkBlock)
k_validate_lds(int64_t N, int C, Model m, const int* __restrict__ pm_cam,
               const int* __restrict__ pm_pt, const float2* __restrict__ xy,
               const float* __restrict__ depth, const double* __restrict__ pts,
               const Cam<double>* __restrict__ camd, const int* __restrict__ inv_cm,
               uint8_t* __restrict__ vrow, uint8_t* __restrict__ vrow_cm) {
  extern __shared__ double lds_cam[];   // C records
  const Cam<double>* tab = stage_cams<kLdsWalkBlock>(camd, C, lds_cam);
  const int64_t stride = int64_t(gridDim.x) * kLdsWalkBlock;
  for (int64_t k = int64_t(blockIdx.x) * kLdsWalkBlock + threadIdx.x; k < N; k += stride) {
    const Cam<double> cm = tab[pm_cam[k]];
    const int p = pm_pt[k];
    double Xc[3];
    cam_frame(cm, pts[3 * p], pts[3 * p + 1], pts[3 * p + 2], Xc);
    bool ok = Xc[2] > m.min_depth;
    if (ok) {
      const double u = cm.f * Xc[0] / Xc[2] + cm.cx;
      const double v = cm.f * Xc[1] / Xc[2] + cm.cy;
      ok = u >= 0.0 && u < double(m.img_w) && v >= 0.0 && v < double(m.img_h);
      if (ok && m.filter_px > 0.0) {
        double e[3];
        residual(cm, Xc, xy[k], 0.0f, 0.0, e);
        ok = e[0] * e[0] + e[1] * e[1] <= m.filter_px * m.filter_px;
      }
    }
    const int rows = 2 + ((m.lam_d > 0.0 && depth[k] > 0.0f) ? 1 : 0);
    const uint8_t v = ok ? uint8_t(rows) : uint8_t(0);
    vrow[k] = v;
    vrow_cm[inv_cm[k]] = v;
  }
}

__global__ void __launch_bounds__(kBlock)
k_cam_rows(const int* __restrict__ cm_off, const uint8_t* __restrict__ vrow_cm,
           const uint8_t* __restrict__ fixed, int need, uint8_t* __restrict__ act_c) {
  __shared__ int smem[kBlock / kWave];
  const int c = blockIdx.x;
  int sum[1] = {0};
  for (int i = cm_off[c] + threadIdx.x; i < cm_off[c + 1]; i += blockDim.x)
    sum[0] += vrow_cm[i];
  block_sum<int, 1>(sum, smem);
  if (threadIdx.x == 0) act_c[c] = (sum[0] >= need && !fixed[c]) ? 1 : 0;
}

// One round of the activity fixpoint on the point side: point rows from the current
// observations, then drop observations whose point is inactive or whose free camera is.
__global__ void __launch_bounds__(kBlock)
k_point_rows_prune(int P, const int* __restrict__ pt_off, const int* __restrict__ pm_cam,
                   const uint8_t* __restrict__ act_c, const uint8_t* __restrict__ fixed,
                   int need, const int* __restrict__ inv_cm, uint8_t* __restrict__ vrow,
                   uint8_t* __restrict__ vrow_cm, uint8_t* __restrict__ act_p,
                   int* __restrict__ changed) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int b = pt_off[p], e = pt_off[p + 1];
  int rows = 0;
  for (int k = b; k < e; ++k) rows += vrow[k];
  const bool a = rows >= need;
  act_p[p] = a ? 1 : 0;
  bool drop = false;
  for (int k = b; k < e; ++k) {
    if (!vrow[k]) continue;
    const int c = pm_cam[k];
    if (!a || !(act_c[c] || fixed[c])) {
      vrow[k] = 0;
      vrow_cm[inv_cm[k]] = 0;
      drop = true;
    }
  }
  if (drop) *changed = 1;   // every writer stores the same value
}

// ------------------------------------------------------------------ compaction kernels
__global__ void __launch_bounds__(kBlock)
k_compact_points(int P, const uint8_t* __restrict__ act_p, const int* __restrict__ rank_p,
                 const int* __restrict__ pt_off, const int* __restrict__ pos_pm,
                 const double* __restrict__ pts, int* __restrict__ pt_src,
                 int* __restrict__ off_hat, double* __restrict__ Xd, float* __restrict__ Xf) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P || !act_p[p]) return;
  const int r = rank_p[p];
  pt_src[r] = p;
  // start and end of the point's compact segment; neighbours store identical values
  off_hat[r] = pos_pm[pt_off[p]];
  off_hat[r + 1] = pos_pm[pt_off[p + 1]];
  for (int i = 0; i < 3; ++i) {
    Xd[3 * r + i] = pts[3 * p + i];
    Xf[3 * r + i] = float(pts[3 * p + i]);
  }
}

__global__ void __launch_bounds__(kBlock)
k_compact_cams(int C, const uint8_t* __restrict__ act_c, const int* __restrict__ rank_c,
               const uint8_t* __restrict__ fixed, const int* __restrict__ fixed_rank,
               const int* __restrict__ cm_off, const int* __restrict__ pos_cm,
               int* __restrict__ slot_all, int* __restrict__ cam_src,
               int* __restrict__ cm_off_hat) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  if (act_c[c]) {
    const int s = rank_c[c];
    slot_all[c] = s;
    cam_src[s] = c;
    cm_off_hat[s] = pos_cm[cm_off[c]];
    cm_off_hat[s + 1] = pos_cm[cm_off[c + 1]];
  } else if (fixed[c]) {
    const int s = rank_c[C] + fixed_rank[c];   // fixed cameras follow the active ones
    slot_all[c] = s;
    cam_src[s] = c;
  } else {
    slot_all[c] = -1;
  }
}

__global__ void __launch_bounds__(kBlock)
k_compact_cam_table(int n, const int* __restrict__ cam_src, const Cam<double>* __restrict__ camd,
                    const Cam<float>* __restrict__ camf, Cam<double>* __restrict__ camd_hat,
                    Cam<float>* __restrict__ camf_hat) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int c = cam_src[s];
  camd_hat[s] = camd[c];
  camf_hat[s] = camf[c];
}

__global__ void __launch_bounds__(kBlock)
k_compact_obs(int64_t N, const uint8_t* __restrict__ vrow, const int* __restrict__ pos_pm,
              const int* __restrict__ pm_cam, const int* __restrict__ slot_all,
              const float2* __restrict__ pm_xy, const float* __restrict__ pm_depth,
              const int* __restrict__ pm_orig, int Ca, const int* __restrict__ inv_cm,
              const int* __restrict__ pos_cm, const int* __restrict__ pm_pt,
              const int* __restrict__ rank_p, int* __restrict__ cam_hat,
              float2* __restrict__ xy_hat, float* __restrict__ depth_hat,
              int* __restrict__ orig_hat, int* __restrict__ pm_cm, int* __restrict__ cm_pt) {
  // XCD x (blockIdx mod 8) takes the x-th eighth of the observations in order, so the scattered
  // camera-major stores of one XCD fill whole lines while they are in its L2 (the grid is a
  // multiple of 8)
  const int per = gridDim.x / 8;
  const int64_t blk = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t k = blk * blockDim.x + threadIdx.x;
  if (k >= N || !vrow[k]) return;
  const int j = pos_pm[k];
  const int slot = slot_all[pm_cam[k]];
  cam_hat[j] = slot;
  if (slot < Ca) {   // solve camera: its camera-major entry and the cross references
    const int i = pos_cm[inv_cm[k]];
    pm_cm[j] = i;
    cm_pt[i] = rank_p[pm_pt[k]];
  } else {
    pm_cm[j] = -1;   // fixed camera: no camera-major entry
  }
  xy_hat[j] = pm_xy[k];
  depth_hat[j] = pm_depth[k];
  orig_hat[j] = pm_orig[k];
}


template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
k_mv_table(int n, const Cam<double>* __restrict__ camd_hat, MvRec<T, D>* __restrict__ mvt) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  MvRec<T, D> v{};
  for (int i = 0; i < 9; ++i) v.R[i] = T(camd_hat[s].R[i]);
  if constexpr (sizeof(T) == 4)
    for (int i = 0; i < 3; ++i) v.c[i] = T(camd_hat[s].c[i]);
  v.f = T(camd_hat[s].f);
  for (int i = 0; i < D; ++i) v.u[i] = T(0);
  mvt[s] = v;
}

// ------------------------------------------------------------------ linearisation
// Workgroup b (XCD-mapped as in the PCG point pass) linearises points [256 b, 256 b + 256) in
// G tiles, with G lanes per point; lanes combine V and gp with shuffles. Partials per
// workgroup: cost, sum |r_2d|^2, max |gp|. With LDS, B = 1024-thread workgroups first copy
// the compact camera table (Ca + Cf records of 120 B) into LDS, so the per-observation camera
// reads hit LDS instead of L2.
template <typename T, bool ADJ, int G, int B, bool LDS>
__global__ void __launch_bounds__(B)
k_lin_point(Model m, Compact<T> cp, ObsMetric<T> om, double* __restrict__ V,
            double* __restrict__ gp, double* __restrict__ partials) {
  __shared__ double smem[3 * (B / kWave)];
  extern __shared__ double lds_cam[];   // LDS: the compact camera table
  const Cam<double>* camtab = cp.camd;
  if constexpr (LDS) camtab = stage_cams<B>(cp.camd, cp.Ca + cp.Cf, lds_cam);
  const int per = gridDim.x / 8;
  const int xcd = blockIdx.x % 8, jw = blockIdx.x / 8;
  const int blk = xcd * per + jw;
  constexpr int tile = B / G;
  const int l = int(threadIdx.x) % G;
  double acc[3] = {0.0, 0.0, 0.0};   // cost, sum |r_2d|^2, max |gp|
  // XCD x owns points [x per B, (x + 1) per B); its workgroups take that range's tiles
  // interleaved (tile t per + jw in the t-th round), so the XCD works on neighbouring tiles
  // and its scattered camera-major stores combine in its L2 (126 us against 143 us with a
  // workgroup's tiles contiguous, 136 us for a persistent grid walking the tiles round-robin;
  // HBM writes 272, 292 and 300 MB on the 1000-camera workload)
  for (int t = 0; t < G; ++t) {
    const int r = xcd * per * B + (t * per + jw) * tile + int(threadIdx.x) / G;
    const bool live = r < cp.Pa;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double g[3] = {0.0, 0.0, 0.0};
    if (live) {
      const double X0 = cp.Xd[3 * r], X1 = cp.Xd[3 * r + 1], X2 = cp.Xd[3 * r + 2];
      const T Xt0 = cp.Xt[3 * r], Xt1 = cp.Xt[3 * r + 1], Xt2 = cp.Xt[3 * r + 2];
      for (int j = cp.off[r] + l; j < cp.off[r + 1]; j += G) {
        const Cam<double> cm = camtab[cp.cam[j]];
        double Xc[3], e[3];
        cam_frame(cm, X0, X1, X2, Xc);
        residual(cm, Xc, cp.xy[j], cp.depth[j], m.lam_d, e);
        const double s = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
        double rho, w, d2;
        huber(s, m.huber, rho, w, d2);
        acc[0] += 0.5 * rho;
        acc[1] += e[0] * e[0] + e[1] * e[1];
        om.w[j] = T(w);
        // the Jacobian streams carry X_c formed in T from the T tables, as the PCG point pass
        // and back-substitution form it
        T Rt[9], ct[3], Xct[3];
#pragma unroll
        for (int i = 0; i < 9; ++i) Rt[i] = T(cm.R[i]);
#pragma unroll
        for (int i = 0; i < 3; ++i) ct[i] = T(cm.c[i]);
        frame_t(Rt, ct, Xt0, Xt1, Xt2, Xct);
        V4<T> xw;
        xw.x = Xct[0];
        xw.y = Xct[1];
        xw.z = Xct[2];
        xw.w = T(w);
        if (om.pm_xcw) om.pm_xcw[j] = xw;
        const int ic = cp.pm_cm[j];   // camera-major copies (solve cameras only)
        if (ic >= 0) {
          om.xcw[ic] = xw;
          V4<T> ev;
          ev.x = T(e[0]);
          ev.y = T(e[1]);
          ev.z = T(e[2]);
          ev.w = T(0);
          om.cm_e[ic] = ev;
        }
        // point block and gradient from float64 rows in both precisions: the depth direction
        // of a weakly observed point can sit below float32 resolution
        AMat<double, ADJ> A;
        A.set(cm.f, m.lam_d, Xc);
        if constexpr (ADJ) {
          const double inv = d2 != 0.0 ? 1.0 / sqrt(s) : 0.0;
          const double eh[3] = {e[0] * inv, e[1] * inv, e[2] * inv};
          om.eh[3 * j] = T(eh[0]);
          om.eh[3 * j + 1] = T(eh[1]);
          om.eh[3 * j + 2] = T(eh[2]);
          if (ic >= 0) {
            om.cm_eh[3 * ic] = T(eh[0]);
            om.cm_eh[3 * ic + 1] = T(eh[1]);
            om.cm_eh[3 * ic + 2] = T(eh[2]);
          }
          if (om.ce) {   // full Hessian: c = rho' e, and V += R^T S R (float64 here)
            const double c3[3] = {w * e[0], w * e[1], w * e[2]};
#pragma unroll
            for (int i = 0; i < 3; ++i) om.ce[3 * j + i] = T(c3[i]);
            if (ic >= 0) {
#pragma unroll
              for (int i = 0; i < 3; ++i) om.cm_ce[3 * ic + i] = T(c3[i]);
            }
            Curv<double> K;
            K.set(cm.f, m.lam_d, Xc, c3);
#pragma unroll
            for (int q = 0; q < 3; ++q) {   // column q of R, then S times it
              const double rq[3] = {cm.R[q], cm.R[3 + q], cm.R[6 + q]};
              double sr[3] = {0.0, 0.0, 0.0};
              K.add_s(rq, sr);
#pragma unroll
              for (int p2 = 0; p2 <= q; ++p2)
                v[sym3(p2, q)] += cm.R[p2] * sr[0] + cm.R[3 + p2] * sr[1] + cm.R[6 + p2] * sr[2];
            }
          }
          A.project(eh);
        }
  #pragma unroll
        for (int i = 0; i < 3; ++i) {
          double a[3], jp[3];
          A.row(i, a);
          rot_tmul(cm, a, jp);
  #pragma unroll
          for (int p = 0; p < 3; ++p) {
  #pragma unroll
            for (int q = p; q < 3; ++q) v[sym3(p, q)] += w * jp[p] * jp[q];
          }
          if constexpr (!ADJ) {
            const double we = w * e[i];
            g[0] += we * jp[0];
            g[1] += we * jp[1];
            g[2] += we * jp[2];
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = group_sum<G>(v[i]);
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = group_sum<G>(g[i]);
    if (live && l == 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) V[6 * r + i] = v[i];
      gp[3 * r] = g[0];
      gp[3 * r + 1] = g[1];
      gp[3 * r + 2] = g[2];
      acc[2] = fmax(acc[2], fmax(fabs(g[0]), fmax(fabs(g[1]), fabs(g[2]))));
    }
  }
  // block reduction: two sums and one max
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  acc[0] = wave_sum(acc[0]);
  acc[1] = wave_sum(acc[1]);
  acc[2] = wave_max(acc[2]);
  if (lane == 0) {
    smem[3 * wid] = acc[0];
    smem[3 * wid + 1] = acc[1];
    smem[3 * wid + 2] = acc[2];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int w = 0; w < int(blockDim.x) / kWave; ++w) {
      a0 += smem[3 * w];
      a1 += smem[3 * w + 1];
      a2 = fmax(a2, smem[3 * w + 2]);
    }
    partials[3 * blk] = a0;
    partials[3 * blk + 1] = a1;
    partials[3 * blk + 2] = a2;
  }
}

// Damped 3x3 point block, inverted in float64 by cofactors.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_point_damp(int Pa, double lam, double dmin, double dmax, const double* __restrict__ V,
             const double* __restrict__ gp, const double* __restrict__ rhs_p,
             T* __restrict__ Vinv, double* __restrict__ hp, PtRec<T>* __restrict__ prec,
             int* __restrict__ bad) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= Pa) return;
  double v00 = V[6 * r], v01 = V[6 * r + 1], v02 = V[6 * r + 2];
  double v11 = V[6 * r + 3], v12 = V[6 * r + 4], v22 = V[6 * r + 5];
  v00 += lam * fmin(fmax(v00, dmin), dmax);
  v11 += lam * fmin(fmax(v11, dmin), dmax);
  v22 += lam * fmin(fmax(v22, dmin), dmax);
  const double c00 = v11 * v22 - v12 * v12;
  const double c01 = v02 * v12 - v01 * v22;
  const double c02 = v01 * v12 - v02 * v11;
  const double c11 = v00 * v22 - v02 * v02;
  const double c12 = v01 * v02 - v00 * v12;
  const double c22 = v00 * v11 - v01 * v01;
  const double det = v00 * c00 + v01 * c01 + v02 * c02;
  double inv[6] = {0, 0, 0, 0, 0, 0};
  if (det > 0.0 && isfinite(det)) {
    const double id = 1.0 / det;
    inv[0] = c00 * id; inv[1] = c01 * id; inv[2] = c02 * id;
    inv[3] = c11 * id; inv[4] = c12 * id; inv[5] = c22 * id;
  } else {
    *bad = 1;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) Vinv[6 * r + i] = T(inv[i]);
  double b[3];
  for (int i = 0; i < 3; ++i) b[i] = rhs_p ? rhs_p[3 * r + i] : -gp[3 * r + i];
  PtRec<T> rec;
  rec.hp[0] = inv[0] * b[0] + inv[1] * b[1] + inv[2] * b[2];
  rec.hp[1] = inv[1] * b[0] + inv[3] * b[1] + inv[4] * b[2];
  rec.hp[2] = inv[2] * b[0] + inv[4] * b[1] + inv[5] * b[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) hp[3 * r + i] = rec.hp[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) rec.vinv[i] = T(inv[i]);
  prec[r] = rec;
}

// D x D SPD inverse through Cholesky (float64); returns false if not positive definite.
template <int D>
__device__ bool spd_inverse(const double* A, double* out) {
  double L[D][D];
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) L[i][j] = 0.0;
  for (int j = 0; j < D; ++j) {
    double d = A[symd<D>(j, j)];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0) || !isfinite(d)) return false;
    const double ljj = sqrt(d);
    L[j][j] = ljj;
    for (int i = j + 1; i < D; ++i) {
      double s = A[symd<D>(i, j)];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      L[i][j] = s / ljj;
    }
  }
  // inverse of L (lower triangular), then A^-1 = L^-T L^-1
  double Li[D][D];
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) Li[i][j] = 0.0;
  for (int j = 0; j < D; ++j) {
    Li[j][j] = 1.0 / L[j][j];
    for (int i = j + 1; i < D; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i][k] * Li[k][j];
      Li[i][j] = -s / L[i][i];
    }
  }
  for (int i = 0; i < D; ++i)
    for (int j = i; j < D; ++j) {
      double s = 0.0;
      for (int k = j; k < D; ++k) s += Li[k][i] * Li[k][j];
      out[symd<D>(i, j)] = s;
    }
  return true;
}


// Workgroup size of the camera-major item kernels: one wave in float32 (an item averages some
// 650 positions on the 1000-camera workload; the PCG camera pass takes 26.0 us against 26.6 us
// with two), two in float64 (58.3 us against 62.5 us with one).
template <typename T>
constexpr int cam_block() {
  return sizeof(T) == 4 ? 64 : 128;
}

// The camera assembly over the camera-pass items, whose positions lie in one XCD's point
// range, so the point records each position gathers stay in that XCD's L2: k_cam_items<SCHUR>
// sums an item's Schur-product rows (sum W Vinv W^T and sum W hp, from the gathered records),
// k_cam_items<!SCHUR> its U and g_c rows (streams only; the two sets of sums in one kernel
// need over 200 VGPRs), and k_cam_assemble adds a camera's item rows in item order and forms
// U*, S_cc, its inverse and the right-hand side. On the 1000-camera workload: one workgroup
// per camera gathering every record from HBM read 3.3x the algorithmic bytes (529 MB,
// 127 us); U and g_c streamed per camera took 66 us, bound by its largest camera (14,000
// observations against a mean of 4,000); both item passes in one kernel, one after the other,
// 141 us (the second pass fetched the streams again).

// The camera-point block of one observation, W = sum over its residual rows of w jc jp^T
// (D x 3), plus the full-Hessian camera-point terms in ADJ mode with curvature.
template <typename T, bool ADJ, int D>
__device__ __forceinline__ void cam_point_block(const Model& m, const Cam<double>& cm,
                                                const ObsMetric<T>& om, int i, const V4<T>& xw,
                                                T (&W)[3 * D]) {
  const T wt = xw.w;
  const T Xt[3] = {xw.x, xw.y, xw.z};
  AMat<T, ADJ> A;
  A.set(T(cm.f), T(m.lam_d), Xt);
  if constexpr (ADJ) A.project(om.cm_eh + 3 * i);
#pragma unroll
  for (int q = 0; q < 3 * D; ++q) W[q] = T(0);
  const T fcol[3] = {Xt[0] / Xt[2], Xt[1] / Xt[2], T(0)};
#pragma unroll
  for (int row = 0; row < 3; ++row) {
    T a[3], jc[D], jp[3];
    A.row(row, a);
    jc[0] = a[0]; jc[1] = a[1]; jc[2] = a[2];
    cross3(Xt, a, jc + 3);
    if constexpr (D == 7) jc[6] = fcol[row];
    rot_tmul(cm, a, jp);
#pragma unroll
    for (int p = 0; p < D; ++p) {
#pragma unroll
      for (int q = 0; q < 3; ++q) W[3 * p + q] += wt * jc[p] * jp[q];
    }
  }
  if constexpr (ADJ) {
    if (om.cm_ce) {   // full Hessian: J_c^T S R + [0 ; -[a]x R] (see Curv)
      const T c3[3] = {om.cm_ce[3 * i], om.cm_ce[3 * i + 1], om.cm_ce[3 * i + 2]};
      Curv<T> K;
      K.set(T(cm.f), T(m.lam_d), Xt, c3);
      T Jc[6][3];   // columns of dX_c / d(rho, phi): e_k, then e_k x X
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T ek[3] = {T(k == 0), T(k == 1), T(k == 2)};
        Jc[k][0] = ek[0]; Jc[k][1] = ek[1]; Jc[k][2] = ek[2];
        cross3(ek, Xt, Jc[3 + k]);
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const T rq[3] = {T(cm.R[q]), T(cm.R[3 + q]), T(cm.R[6 + q])};
        T sr[3] = {T(0), T(0), T(0)};
        K.add_s(rq, sr);
        T axr[3];
        cross3(K.a, rq, axr);
#pragma unroll
        for (int p = 0; p < 6; ++p)
          W[3 * p + q] += Jc[p][0] * sr[0] + Jc[p][1] * sr[1] + Jc[p][2] * sr[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) W[3 * (3 + k) + q] -= axr[k];
      }
    }
  }
}

// Per item, rows [0, NS) sum W Vinv W^T and [NS, NS + D) sum W hp (SCHUR), or rows
// [NS + D, 2 NS + D) U and [2 NS + D, 2 NS + 2 D) g_c (zero in ADJ mode), into
// part[item * 2 (NS + D) + row] (item-major: one contiguous write per item, and a camera's
// items are adjacent). The SCHUR kernel loads the next position's stream entry and point
// record while this one is summed (and the point rank two positions ahead).
template <int D>
constexpr int cam_item_rows() {
  return 2 * (sym_count(D) + D);
}

template <typename T, bool ADJ, int D, bool SCHUR>
__global__ void __launch_bounds__(cam_block<T>())
k_cam_items(Model m, Compact<T> cp, ObsMetric<T> om, const PtRec<T>* __restrict__ prec,
            CamItems it, double* __restrict__ part) {
  constexpr int NS = sym_count(D);
  constexpr int KA = NS + D;
  constexpr int B = cam_block<T>();
  __shared__ double smem[KA * (B / kWave)];
  const int4 rec = it.at[(blockIdx.x % it.R) * it.cap + blockIdx.x / it.R];
  if (rec.x < 0) return;   // past the range's last item
  const Cam<double> cm = cp.camd[rec.y];
  double acc[KA];
#pragma unroll
  for (int q = 0; q < KA; ++q) acc[q] = 0.0;
  if constexpr (SCHUR) {
    const int i1 = rec.w;
    int i = rec.z + int(threadIdx.x);
    V4<T> xwn{};
    PtRec<T> prn{};
    if (i < i1) {
      xwn = om.xcw[i];
      prn = prec[cp.cm_pt[i]];
    }
    int pn = i + B < i1 ? cp.cm_pt[i + B] : 0;
    for (; i < i1; i += B) {
      const V4<T> xw = xwn;
      const PtRec<T> pr = prn;
      if (i + B < i1) {
        xwn = om.xcw[i + B];
        prn = prec[pn];
        pn = i + 2 * B < i1 ? cp.cm_pt[i + 2 * B] : 0;
      }
      T W[3 * D];
      cam_point_block<T, ADJ, D>(m, cm, om, i, xw, W);
      T vi[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) vi[q] = pr.vinv[q];
      T WV[3 * D];
#pragma unroll
      for (int p = 0; p < D; ++p) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
          WV[3 * p + q] = W[3 * p] * vi[sym3(0, q)] + W[3 * p + 1] * vi[sym3(1, q)] +
                          W[3 * p + 2] * vi[sym3(2, q)];
        acc[NS + p] += double(W[3 * p]) * pr.hp[0] + double(W[3 * p + 1]) * pr.hp[1] +
                       double(W[3 * p + 2]) * pr.hp[2];
      }
#pragma unroll
      for (int p = 0; p < D; ++p) {
#pragma unroll
        for (int q = p; q < D; ++q)
          acc[symd<D>(p, q)] += double(WV[3 * p] * W[3 * q] + WV[3 * p + 1] * W[3 * q + 1] +
                                       WV[3 * p + 2] * W[3 * q + 2]);
      }
    }
  }
  // U in T per lane (the J^T J blocks are float32 in mixed precision), g_c in float64; the
  // next position's stream entries are loaded while this one is summed
  T U[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) U[q] = T(0);
  if constexpr (!SCHUR) {
    const int i1 = rec.w;
    int i = rec.z + int(threadIdx.x);
    V4<T> xwn{}, evn{};
    if (i < i1) {
      xwn = om.xcw[i];
      if constexpr (!ADJ) evn = om.cm_e[i];
    }
    for (; i < i1; i += B) {
      const V4<T> xw = xwn;
      const V4<T> ev = evn;
      if (i + B < i1) {
        xwn = om.xcw[i + B];
        if constexpr (!ADJ) evn = om.cm_e[i + B];
      }
      const T wt = xw.w;
      const T Xt[3] = {xw.x, xw.y, xw.z};
      AMat<T, ADJ> A;
      A.set(T(cm.f), T(m.lam_d), Xt);
      if constexpr (ADJ) A.project(om.cm_eh + 3 * i);
      const double e[3] = {double(ev.x), double(ev.y), double(ev.z)};
      double g6[D];
#pragma unroll
      for (int q = 0; q < D; ++q) g6[q] = 0.0;
      // de/df of the pinhole rows (focal length as the seventh unknown)
      const T fcol[3] = {Xt[0] / Xt[2], Xt[1] / Xt[2], T(0)};
#pragma unroll
      for (int row = 0; row < 3; ++row) {
        T a[3], jc[D];
        A.row(row, a);
        jc[0] = a[0]; jc[1] = a[1]; jc[2] = a[2];
        cross3(Xt, a, jc + 3);
        if constexpr (D == 7) jc[6] = fcol[row];
#pragma unroll
        for (int p = 0; p < D; ++p) {
#pragma unroll
          for (int q = p; q < D; ++q) U[symd<D>(p, q)] += wt * jc[p] * jc[q];
        }
        if constexpr (!ADJ) {
          const double we = double(wt) * e[row];
#pragma unroll
          for (int p = 0; p < D; ++p) g6[p] += we * double(jc[p]);
        }
      }
      if constexpr (ADJ) {
        if (om.cm_ce) {   // full Hessian: the curvature and retraction terms (see Curv)
          const T c3[3] = {om.cm_ce[3 * i], om.cm_ce[3 * i + 1], om.cm_ce[3 * i + 2]};
          Curv<T> Kc;
          Kc.set(T(cm.f), T(m.lam_d), Xt, c3);
          // columns of dX_c / d(rho, phi): e_k, then e_k x X
          T Jc[6][3];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const T ek[3] = {T(k == 0), T(k == 1), T(k == 2)};
            Jc[k][0] = ek[0]; Jc[k][1] = ek[1]; Jc[k][2] = ek[2];
            cross3(ek, Xt, Jc[3 + k]);
          }
          T SJ[6][3];
#pragma unroll
          for (int p = 0; p < 6; ++p) {
            SJ[p][0] = SJ[p][1] = SJ[p][2] = T(0);
            Kc.add_s(Jc[p], SJ[p]);
          }
#pragma unroll
          for (int p = 0; p < 6; ++p) {
#pragma unroll
            for (int q = p; q < 6; ++q)
              U[symd<D>(p, q)] += Jc[p][0] * SJ[q][0] + Jc[p][1] * SJ[q][1] + Jc[p][2] * SJ[q][2];
          }
          // retraction terms: rho-phi [a]x / 2, phi-phi (a X^T + X a^T) / 2 - (a.X) I
          const T* a = Kc.a;
          const T ax[3][3] = {{T(0), -a[2], a[1]}, {a[2], T(0), -a[0]}, {-a[1], a[0], T(0)}};
          const T aX = a[0] * Xt[0] + a[1] * Xt[1] + a[2] * Xt[2];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int l = 0; l < 3; ++l) U[symd<D>(k, 3 + l)] += T(0.5) * ax[k][l];
#pragma unroll
            for (int l = k; l < 3; ++l)
              U[symd<D>(3 + k, 3 + l)] +=
                  T(0.5) * (a[k] * Xt[l] + Xt[k] * a[l]) - (k == l ? aX : T(0));
          }
        }
      }
#pragma unroll
      for (int p = 0; p < D; ++p) acc[NS + p] += g6[p];
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) acc[q] = double(U[q]);
  }
  block_sum<double, KA>(acc, smem);
  if (threadIdx.x == 0) {
    double* row = part + size_t(rec.x) * (2 * KA) + (SCHUR ? 0 : KA);
#pragma unroll
    for (int q = 0; q < KA; ++q) row[q] = acc[q];
  }
}

// Per camera slot: the camera's item rows added in item order (lane group g takes items g,
// g + kG, ..., then each row over the groups), then U* = U + lam diag, S_cc = U* - sum W Vinv
// W^T and its inverse, b = rhs_c - sum W hp (rhs_c = -g_c unless given).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
k_cam_assemble(int Ca, double lam, double dmin, double dmax, const int* __restrict__ item_off,
               const double* __restrict__ part, const double* __restrict__ rhs_c,
               double* __restrict__ Uraw, T* __restrict__ Ustar, double* __restrict__ gc,
               double* __restrict__ b, double* __restrict__ Minv, double* __restrict__ Scc) {
  constexpr int NS = sym_count(D);
  constexpr int KR = cam_item_rows<D>();
  constexpr int kG = kBlock / KR;
  static_assert(kG >= 1, "one row per thread");
  __shared__ double s_rows[kG][KR];
  __shared__ double s_tot[KR];
  const int s = blockIdx.x;
  {
    const int q = int(threadIdx.x) % KR, g = int(threadIdx.x) / KR;
    if (g < kG) {
      double a = 0.0;
      for (int it = item_off[s] + g; it < item_off[s + 1]; it += kG)
        a += part[size_t(it) * KR + q];
      s_rows[g][q] = a;
    }
    __syncthreads();
    if (int(threadIdx.x) < KR) {
      double a = s_rows[0][threadIdx.x];
      for (int h = 1; h < kG; ++h) a += s_rows[h][threadIdx.x];
      s_tot[threadIdx.x] = a;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double* S = s_tot;                 // sum W Vinv W^T
  const double* Wh = s_tot + NS;           // sum W hp
  const double* U = s_tot + NS + D;        // J_c^T M J_c
  const double* g = s_tot + 2 * NS + D;    // g_c
  double Us[NS], Sc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    Uraw[NS * s + q] = U[q];
    Us[q] = U[q];
  }
#pragma unroll
  for (int p = 0; p < D; ++p) {
    const int d = symd<D>(p, p);
    Us[d] += lam * fmin(fmax(U[d], dmin), dmax);
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    Ustar[q * Ca + s] = T(Us[q]);
    Sc[q] = Us[q] - S[q];
    if (Scc) Scc[q * Ca + s] = Sc[q];
  }
#pragma unroll
  for (int p = 0; p < D; ++p) {
    gc[p * Ca + s] = g[p];
    const double rhs = rhs_c ? rhs_c[p * Ca + s] : -g[p];
    b[p * Ca + s] = rhs - Wh[p];
  }
  double inv[NS];
  if (!spd_inverse<D>(Sc, inv)) {
    // block not positive definite (rounding at tiny damping): Jacobi fallback on U*
#pragma unroll
    for (int q = 0; q < NS; ++q) inv[q] = 0.0;
#pragma unroll
    for (int p = 0; p < D; ++p) {
      const double d = Us[symd<D>(p, p)];
      inv[symd<D>(p, p)] = d > 0.0 ? 1.0 / d : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) Minv[q * Ca + s] = inv[q];
}

// ------------------------------------------------------------------ PCG
// y = M x for a symmetric D x D block stored SoA (D (D + 1) / 2 arrays of length Ca).
template <int D>
__device__ __forceinline__ void symd_mul_soa(const double* M, int Ca, int s, const double* x,
                                             double* y) {
  double m[sym_count(D)];
#pragma unroll
  for (int k = 0; k < sym_count(D); ++k) m[k] = M[k * Ca + s];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) a += m[symd<D>(i, j)] * x[j];
    y[i] = a;
  }
}

// One thread per camera and range r >= 1: the first position of the camera's segment (sorted
// by point rank) whose rank is at least r * ppx, by binary search.
__global__ void __launch_bounds__(kBlock)
k_range_bounds(int Ca, int R, int ppx, const int* __restrict__ cm_off,
               const int* __restrict__ cm_pt, int* __restrict__ rb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Ca * R) return;
  const int r = t / Ca, s = t % Ca;
  int lo = cm_off[s], hi = cm_off[s + 1];
  if (r > 0) {
    const int64_t key = int64_t(r) * ppx;
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      if (cm_pt[mid] < key)
        lo = mid + 1;
      else
        hi = mid;
    }
  }
  rb[t] = lo;
}

// Builds the items of the camera passes (see CamItems): R + 1 exclusive scans over the
// cameras in tiles of the block, of each camera's item count (numbering camera by camera) and
// of its count in every range (the per-range lists). One workgroup of 1024 threads.
__global__ void __launch_bounds__(1024)
k_build_items(int Ca, const int* __restrict__ cm_off, const int* __restrict__ rb, int K,
              CamItems it) {
  constexpr int NV = kMaxRanges + 1;
  __shared__ int s_wave[NV][1024 / kWave];
  __shared__ int s_carry[NV];
  const int R = it.R;
  if (threadIdx.x < NV) s_carry[threadIdx.x] = 0;
  for (int q = threadIdx.x; q < R * it.cap; q += blockDim.x) it.at[q] = make_int4(-1, 0, 0, 0);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int base = 0; base < Ca; base += 1024) {
    const int s = base + int(threadIdx.x);
    int lo[kMaxRanges + 1], cnt[NV], incl[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) cnt[v] = 0;
    if (s < Ca) {
#pragma unroll
      for (int q = 0; q < kMaxRanges; ++q)
        if (q < R) lo[q] = q == 0 ? cm_off[s] : rb[q * Ca + s];
      const int end = cm_off[s + 1];
#pragma unroll
      for (int q = 0; q < kMaxRanges; ++q) {
        if (q < R) {
          const int hi = q + 1 < R ? lo[q + 1] : end;
          cnt[1 + q] = (hi - lo[q] + K - 1) / K;
          cnt[0] += cnt[1 + q];
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      incl[v] = cnt[v];
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(incl[v], o, kWave);
        if (lane >= o) incl[v] += t;
      }
      if (lane == kWave - 1) s_wave[v][wid] = incl[v];
    }
    __syncthreads();
    int first[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      int before = s_carry[v];
      for (int w = 0; w < wid; ++w) before += s_wave[v][w];
      first[v] = before + incl[v] - cnt[v];
    }
    if (s < Ca) {
      it.off[s] = first[0];
      int i = first[0];
      const int end = cm_off[s + 1];
#pragma unroll
      for (int q = 0; q < kMaxRanges; ++q) {
        if (q < R) {
          const int hi = q + 1 < R ? lo[q + 1] : end;
          for (int c = 0; c < cnt[1 + q]; ++c, ++i)
            it.at[q * it.cap + first[1 + q] + c] =
                make_int4(i, s, lo[q] + c * K, min(lo[q] + (c + 1) * K, hi));
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 1023) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s_carry[v] = first[v] + cnt[v];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    it.off[Ca] = s_carry[0];
    int mx = 0;
    for (int q = 0; q < R; ++q) mx = max(mx, s_carry[1 + q]);
    it.off[Ca + 1] = mx;
  }
}

template <typename T, int D>
__global__ void __launch_bounds__(1024)
k_pcg_init(int Ca, const double* __restrict__ b, const double* __restrict__ Minv,
           const T* __restrict__ Ustar, double* __restrict__ x,
           double* __restrict__ r, double* __restrict__ u, double* __restrict__ p,
           double* __restrict__ sv, double* __restrict__ Uu, double* __restrict__ terms,
           MvRec<T, D>* __restrict__ mvt, PcgState* st, double tol2, int max_iter) {
  __shared__ double smem[1024 / kWave];
  double acc[1] = {0.0};   // b.b
  for (int s = threadIdx.x; s < Ca; s += blockDim.x) {
    double rv[D], uv[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      rv[i] = b[i * Ca + s];
      x[i * Ca + s] = 0.0;
      r[i * Ca + s] = rv[i];
      p[i * Ca + s] = 0.0;
      sv[i * Ca + s] = 0.0;
      acc[0] += rv[i] * rv[i];
    }
    symd_mul_soa<D>(Minv, Ca, s, rv, uv);
    double ru = 0.0, uUu = 0.0, rr = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      u[i * Ca + s] = uv[i];
      mvt[s].u[i] = T(uv[i]);
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) a += double(Ustar[symd<D>(i, j) * Ca + s]) * uv[j];
      Uu[i * Ca + s] = a;
      ru += rv[i] * uv[i];
      uUu += uv[i] * a;
      rr += rv[i] * rv[i];
    }
    terms[s] = ru;
    terms[Ca + s] = uUu;
    terms[2 * Ca + s] = rr;
  }
  block_sum<double, 1>(acc, smem);
  if (threadIdx.x == 0) {
    st->gam[0] = st->gam[1] = 0.0;
    st->alp[0] = st->alp[1] = 0.0;
    st->bb = acc[0];
    st->rr = acc[0];
    st->tol2 = tol2;
    st->iter = 0;
    st->matvecs = 0;
    st->max_iter = max_iter;
    st->breakdown = 0;
    st->done = (acc[0] == 0.0 || max_iter <= 0) ? 1 : 0;
    if (!isfinite(acc[0])) {
      st->breakdown = 1;
      st->done = 1;
    }
  }
}

// Point-major pass of S u: G lanes share one point, each walks every G-th observation of
// the point's segment, and the lanes combine their sums with shuffles (G divides 64). Per
// observation: its camera slot and the matvec record of its camera (R, c, f, u). In float32
// the observation adds its weight w and X_c = R (X - c) is formed from the point, read once
// per point; in float64 it streams the stored (X_c, w) 4-vector (forming X_c there costs
// more in float64 arithmetic and in 160-byte records than the 24 bytes it saves).
// The point's z = Vinv y is then stored at the camera-major position of each of its
// observations, so that the camera pass streams z instead of gathering it.

// What a lane needs before it can start on its point: the point's observation range and
// coordinates, and its own first observation (camera slot, weight, camera-major position).
// The persistent pass loads these one tile ahead, so that a tile starts on data already in
// registers instead of waiting on the chain offsets -> slot -> record.
template <typename T>
struct PtLoad {
  int b, e;     // observation range; b = e for a lane without a point
  int s0;       // first observation's camera slot (Ca: none)
  V4<T> xw0;    // its weight in w; in float64 also its X_c (the stored 4-vector)
  T X[3];       // the point (float32)
};
// X_c is formed in the point pass in float32 and streamed in float64.
template <typename T>
constexpr bool kFormXc = sizeof(T) == 4;

// Fills the per-lane part of p for point r; p.b and p.e must be set.
template <typename T>
__device__ __forceinline__ void pt_load_first(const Compact<T>& cp, const ObsMetric<T>& om,
                                              int r, int l, PtLoad<T>& p) {
  p.s0 = cp.Ca;
  p.xw0.x = p.xw0.y = p.xw0.z = p.xw0.w = T(0);
  p.X[0] = p.X[1] = p.X[2] = T(0);
  if (kFormXc<T> && p.b < p.e) {
    p.X[0] = cp.Xt[3 * r];
    p.X[1] = cp.Xt[3 * r + 1];
    p.X[2] = cp.Xt[3 * r + 2];
  }
  if (p.b + l < p.e) {
    p.s0 = cp.cam[p.b + l];
    if constexpr (kFormXc<T>)
      p.xw0.w = om.w[p.b + l];
    else
      p.xw0 = om.pm_xcw[p.b + l];
  }
}

// One observation's term of y_p = sum_k R_k^T W_k (J_c u)_k, added to y: W = w A^T A with A
// the rows of de/dX_c at X_c (projected in the adjoint metric; with the full Hessian, plus the
// curvature and retraction terms of the observation j).
template <typename T, bool ADJ, int D>
__device__ __forceinline__ void point_obs_term(const Model& m, const ObsMetric<T>& om,
                                               const MvRec<T, D>& mc, const T Xc[3], T wj,
                                               int j, T y[3]) {
  AMat<T, ADJ> A;
  A.set(mc.f, T(m.lam_d), Xc);
  if constexpr (ADJ) A.project(om.eh + 3 * j);
  T o3[3], d[3], tt[3], mm[3];
  const T w3[3] = {mc.u[3], mc.u[4], mc.u[5]};
  cross3(w3, Xc, o3);
  d[0] = mc.u[0] + o3[0];
  d[1] = mc.u[1] + o3[1];
  d[2] = mc.u[2] + o3[2];
  A.apply(d, tt);
  if constexpr (D == 7) {   // focal column (x/z, y/z, 0) times the focal unknown
    const T uf = mc.u[6] / Xc[2];
    tt[0] += Xc[0] * uf;
    tt[1] += Xc[1] * uf;
  }
  A.applyT(tt, mm);
  mm[0] *= wj; mm[1] *= wj; mm[2] *= wj;
  if constexpr (ADJ) {
    if (om.ce) {   // full Hessian: + S d + a x u_phi (see Curv)
      const T c3[3] = {om.ce[3 * j], om.ce[3 * j + 1], om.ce[3 * j + 2]};
      Curv<T> K;
      K.set(mc.f, T(m.lam_d), Xc, c3);
      K.add_s(d, mm);
      T au[3];
      cross3(K.a, w3, au);
      mm[0] += au[0]; mm[1] += au[1]; mm[2] += au[2];
    }
  }
  // R^T m
  y[0] += mc.R[0] * mm[0] + mc.R[3] * mm[1] + mc.R[6] * mm[2];
  y[1] += mc.R[1] * mm[0] + mc.R[4] * mm[1] + mc.R[7] * mm[2];
  y[2] += mc.R[2] * mm[0] + mc.R[5] * mm[1] + mc.R[8] * mm[2];
}

// Every lane of a wave must call this together (shuffles); lanes with !live do nothing.
template <typename T, bool ADJ, int G, int D>
__device__ __forceinline__ void schur_point_one(const Model& m, const Compact<T>& cp,
                                                const ObsMetric<T>& om,
                                                const MvRec<T, D>* __restrict__ tab,
                                                const T* __restrict__ Vinv,
                                                P3<T>* __restrict__ zq, int r, bool live,
                                                int l, const PtLoad<T>& p) {
  T y[3] = {T(0), T(0), T(0)};
  T vi[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  // y += R^T W (J_c u) for one observation
  auto obs = [&](int j, int s, const V4<T>& xw) {
    if (s >= cp.Ca) return;   // fixed camera: no column in the solve
    const MvRec<T, D> mc = tab[s];
    T Xc[3];
    if constexpr (kFormXc<T>) {
      frame_t(mc.R, mc.c, p.X[0], p.X[1], p.X[2], Xc);
    } else {
      Xc[0] = xw.x;
      Xc[1] = xw.y;
      Xc[2] = xw.z;
    }
    point_obs_term<T, ADJ, D>(m, om, mc, Xc, xw.w, j, y);
  };
  if (live) {
    // loads needed only after the reduction, issued now to overlap the stream (float32: the
    // registers are free; float64 keeps them for the stream)
    if constexpr (sizeof(T) == 4) {
      if (l == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) vi[q] = Vinv[6 * r + q];
      }
    }
    int j = p.b + l;
    if (j < p.e) {
      obs(j, p.s0, p.xw0);
      for (j += G; j < p.e; j += G) {
        V4<T> xw;
        if constexpr (kFormXc<T>) {
          xw.x = xw.y = xw.z = T(0);
          xw.w = om.w[j];
        } else {
          xw = om.pm_xcw[j];
        }
        obs(j, cp.cam[j], xw);
      }
    }
  }
  y[0] = group_sum<G>(y[0]);
  y[1] = group_sum<G>(y[1]);
  y[2] = group_sum<G>(y[2]);
  // every lane of the group now holds y; the first lane stores the point's z (consecutive
  // groups store consecutive points, so the stores fill whole cache lines)
  if (live && l == 0) {
    if constexpr (sizeof(T) != 4) {
#pragma unroll
      for (int q = 0; q < 6; ++q) vi[q] = Vinv[6 * r + q];
    }
    P3<T> z;
    z.x = vi[0] * y[0] + vi[1] * y[1] + vi[2] * y[2];
    z.y = vi[1] * y[0] + vi[3] * y[1] + vi[4] * y[2];
    z.z = vi[2] * y[0] + vi[4] * y[1] + vi[5] * y[2];
    zq[r] = z;
  }
}

// One thread group per point, matvec records read from global memory (any camera count).
// The grid is a multiple of 8 and consecutive workgroups go to the 8 XCDs in turn; each XCD
// takes one contiguous eighth of the point ranks, so the z stores of one XCD fill whole
// cache lines of every camera segment (segments are sorted by point rank) in its own L2.
template <typename T, bool ADJ, int G, int D>
__global__ void __launch_bounds__(kBlock)
k_schur_point(Model m, Compact<T> cp, ObsMetric<T> om, const MvRec<T, D>* __restrict__ mvt,
              const T* __restrict__ Vinv, P3<T>* __restrict__ zq,
              const PcgState* __restrict__ st) {
  if (st->done) return;
  const int per = gridDim.x / 8;
  const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const int t = blk * blockDim.x + threadIdx.x;
  const int r = t / G, l = t % G;
  const bool live = r < cp.Pa;
  PtLoad<T> p;
  p.b = live ? cp.off[r] : 0;
  p.e = live ? cp.off[r + 1] : 0;
  pt_load_first(cp, om, r, l, p);
  schur_point_one<T, ADJ, G, D>(m, cp, om, mvt, Vinv, zq, r, live, l, p);
}

// Grid-stride variant for tables that fit in LDS: each 1024-thread workgroup copies the camera
// records into LDS once, so the random per-observation record reads hit LDS.
// XCD x owns the x-th eighth of the point ranks (ppx points) and its workgroups take that
// range's tiles round-robin, so the z vectors of a range are written through the L2 of the
// XCD whose camera-pass workgroups read them (CamItems).
// Loads run ahead of the work: the offsets two tiles ahead and, in float32, the next tile's
// first-observation data are issued before the current tile is processed.
constexpr int kPtLdsBlock = 1024;

template <typename T, bool ADJ, int G, int D>
__global__ void __launch_bounds__(kPtLdsBlock)
k_schur_point_lds(Model m, Compact<T> cp, ObsMetric<T> om, const MvRec<T, D>* __restrict__ mvt,
                  const T* __restrict__ Vinv, P3<T>* __restrict__ zq,
                  const PcgState* __restrict__ st, int ppx) {
  extern __shared__ uint4 lds_tab[];   // cp.Ca records
  if (st->done) return;
  const int per = gridDim.x / 8;            // workgroups per XCD
  const int xcd = blockIdx.x % 8;
  const int jw = blockIdx.x / 8;
  const int lo = xcd * ppx;
  const int hi = min(cp.Pa, lo + ppx);
  constexpr int tile = kPtLdsBlock / G;
  const int step = per * tile;
  const int l = int(threadIdx.x) % G;
  int r = lo + jw * tile + int(threadIdx.x) / G;
  PtLoad<T> cur;
  cur.b = r < hi ? cp.off[r] : 0;
  cur.e = r < hi ? cp.off[r + 1] : 0;
  if constexpr (kFormXc<T>) pt_load_first(cp, om, r, l, cur);
  int bn = 0, en = 0;   // offsets of the next tile
  if (r + step < hi) {
    bn = cp.off[r + step];
    en = cp.off[r + step + 1];
  }
  const int nchunk = cp.Ca * int(sizeof(MvRec<T, D>) / sizeof(uint4));
  const uint4* src = reinterpret_cast<const uint4*>(mvt);
  for (int i = threadIdx.x; i < nchunk; i += kPtLdsBlock) lds_tab[i] = src[i];
  __syncthreads();
  const MvRec<T, D>* tab = reinterpret_cast<const MvRec<T, D>*>(lds_tab);
  for (int base = lo + jw * tile; base < hi; base += step, r += step) {
    PtLoad<T> nxt;
    nxt.b = bn;
    nxt.e = en;
    if constexpr (kFormXc<T>)
      pt_load_first(cp, om, r + step, l, nxt);   // float32: one tile ahead
    else
      pt_load_first(cp, om, r, l, cur);          // float64: in the tile (measured faster)
    bn = en = 0;
    if (r + 2 * step < hi) {
      bn = cp.off[r + 2 * step];
      en = cp.off[r + 2 * step + 1];
    }
    schur_point_one<T, ADJ, G, D>(m, cp, om, tab, Vinv, zq, r, r < hi, l, cur);
    cur = nxt;
  }
}

// Camera-major pass of S u over the items of CamItems: a workgroup sums W_k z_k over an item's
// positions into partial i (z gathered by the position's point rank) and writes the partial's
// dot with u_s to the last row. No item has more than K positions whatever the spread of
// observations per camera, and the update kernel adds a camera's partials in item order, so
// the result does not depend on scheduling. Workgroup b takes slot b / R of range b % R: the
// workgroups of XCD r (b % 8 = r) take range r's items, whose z vectors the point pass has
// just written through that XCD's L2 (without the split, 43 us and 2.9x the fetched bytes on
// the 1000-camera workload). Workgroups of cam_block<T>() threads.
constexpr int kCamBlock = 128;   // global-positioning camera pass

// One item of the camera pass (all threads of the workgroup).
template <typename T, bool ADJ, int D>
__device__ __forceinline__ void cam_item(const Model& m, const Compact<T>& cp,
                                         const ObsMetric<T>& om, const double* __restrict__ u,
                                         const P3<T>* __restrict__ zq, int4 rec, int nslot,
                                         double* __restrict__ part, T* smem, int Ca) {
  const int i = rec.x, s = rec.y, sb = rec.z, se = rec.w;
  double us[D];
  if (threadIdx.x == 0) {   // needed after the reduction: loaded while the stream runs
#pragma unroll
    for (int q = 0; q < D; ++q) us[q] = u[q * Ca + s];
  }
  const Cam<T> cm = cp.camt[s];
  T acc[D];
#pragma unroll
  for (int q = 0; q < D; ++q) acc[q] = T(0);
#pragma unroll 4
  for (int k = sb + threadIdx.x; k < se; k += cam_block<T>()) {
    const V4<T> xw = om.xcw[k];
    const P3<T> zv = zq[cp.cm_pt[k]];
    const T Xc[3] = {xw.x, xw.y, xw.z};
    AMat<T, ADJ> A;
    A.set(cm.f, T(m.lam_d), Xc);
    if constexpr (ADJ) A.project(om.cm_eh + 3 * k);
    const T z3[3] = {zv.x, zv.y, zv.z};
    T uu[3], t[3], mm[3], xm[3];
    rot_mul(cm, z3, uu);
    A.apply(uu, t);
    A.applyT(t, mm);
    if constexpr (D == 7)   // focal column: w (x/z, y/z, 0) . t
      acc[6] += xw.w * (Xc[0] * t[0] + Xc[1] * t[1]) / Xc[2];
    mm[0] *= xw.w; mm[1] *= xw.w; mm[2] *= xw.w;
    T ua[3] = {T(0), T(0), T(0)};
    if constexpr (ADJ) {
      if (om.cm_ce) {   // full Hessian: + S (R z), and (R z) x a in the rotation rows
        const T c3[3] = {om.cm_ce[3 * k], om.cm_ce[3 * k + 1], om.cm_ce[3 * k + 2]};
        Curv<T> K;
        K.set(cm.f, T(m.lam_d), Xc, c3);
        K.add_s(uu, mm);
        cross3(uu, K.a, ua);
      }
    }
    cross3(Xc, mm, xm);
    acc[0] += mm[0]; acc[1] += mm[1]; acc[2] += mm[2];
    acc[3] += xm[0] + ua[0]; acc[4] += xm[1] + ua[1]; acc[5] += xm[2] + ua[2];
  }
  block_sum<T, D>(acc, smem);
  if (threadIdx.x == 0) {
    double pd = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const double v = double(acc[q]);
      part[q * nslot + i] = v;
      pd += us[q] * v;
    }
    part[D * nslot + i] = pd;
  }
}

template <typename T, bool ADJ, int D>
__global__ void __launch_bounds__(cam_block<T>())
k_schur_cam(Model m, Compact<T> cp, ObsMetric<T> om, const double* __restrict__ u,
            const P3<T>* __restrict__ zq, CamItems it, int nslot, double* __restrict__ part,
            const PcgState* __restrict__ st) {
  if (st->done) return;
  const int4 rec = it.at[(blockIdx.x % it.R) * it.cap + blockIdx.x / it.R];
  if (rec.x < 0) return;   // past the range's last item
  __shared__ T smem[D * (cam_block<T>() / kWave)];
  cam_item<T, ADJ, D>(m, cp, om, u, zq, rec, nslot, part, smem, cp.Ca);
}

// One Chronopoulos-Gear PCG iteration k after the matvec w = S u, with w_s = U*_s u_s minus the
// camera's item partials:
//   gamma = r.u, delta = w.u = u.U*u - (the items' partial . u), rho = r.r (one reduction);
//   stop if rho <= tol^2 b.b; beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma /
//   alpha_prev); p = u + beta p; s = w + beta s; x += alpha p; r -= alpha s; u = M^-1 r;
//   then U*u and the camera's terms r.u, u.U*u, r.r of the next iteration.
// The per-camera terms are double-buffered by iteration parity, since every workgroup reduces
// all of them (in the same fixed order, so all take the same scalars and the same decision)
// while owners write the next ones. Workgroup 0 records the scalars.
constexpr int kUpdBlock = 512;
constexpr int kUpdCams = 64;
constexpr int kUpdDots = 16;   // item dots per thread loaded at once (8: 8.7 us, 16: 7.7 us)
constexpr int kUpdTerms = 4;   // per-camera terms per thread loaded at once

template <typename T, int D>
__global__ void __launch_bounds__(kUpdBlock)
k_pcg_update(int Ca, int k, const double* __restrict__ Minv, const T* __restrict__ Ustar,
             const int* __restrict__ item_off, int nit, int nslot, const double* __restrict__ part,
             double* __restrict__ terms, double* __restrict__ x, double* __restrict__ r,
             double* __restrict__ u, double* __restrict__ p, double* __restrict__ sv,
             double* __restrict__ Uu, MvRec<T, D>* __restrict__ mvt, PcgState* st) {
  __shared__ double smem[3 * (kUpdBlock / kWave)];
  __shared__ double s_bcast[2];
  __shared__ double s_items[kUpdCams][D];
  __shared__ int s_go;
  const double* tin = terms + (k & 1) * 3 * Ca;
  double* tout = terms + ((k + 1) & 1) * 3 * Ca;
  const int s = blockIdx.x * kUpdCams + threadIdx.x;
  const bool own = threadIdx.x < kUpdCams && s < Ca;
  // every load the owner needs is issued first, then the global sums' and the camera's item
  // partials (summed after the sums: 7.5 us against 7.9 us with the partials first)
  double pv[D], wv[D], sv0[D], rv[D], uv[D], xv[D], m[sym_count(D)];
  T us[sym_count(D)];
  if (own) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      pv[i] = p[i * Ca + s];
      wv[i] = Uu[i * Ca + s];
      sv0[i] = sv[i * Ca + s];
      rv[i] = r[i * Ca + s];
      uv[i] = u[i * Ca + s];
      xv[i] = x[i * Ca + s];
    }
#pragma unroll
    for (int q = 0; q < sym_count(D); ++q) {
      m[q] = Minv[q * Ca + s];
      us[q] = Ustar[q * Ca + s];
    }
  }
  // the per-camera terms and the items' dots, in batches whose loads are all in flight at
  // once; each thread adds its values in index order
  double acc[3] = {0.0, 0.0, 0.0};   // gamma, delta, rho
  for (int c0 = threadIdx.x; c0 < Ca; c0 += kUpdTerms * kUpdBlock) {
    double tt[3][kUpdTerms];
#pragma unroll
    for (int q = 0; q < kUpdTerms; ++q) {
      const int c = c0 + q * kUpdBlock;
#pragma unroll
      for (int k = 0; k < 3; ++k) tt[k][q] = c < Ca ? tin[k * Ca + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kUpdTerms; ++q) {
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[k] += tt[k][q];
    }
  }
  const double* dot = part + size_t(D) * nslot;
  for (int j0 = threadIdx.x; j0 < nit; j0 += kUpdDots * kUpdBlock) {
    double dd[kUpdDots];
#pragma unroll
    for (int q = 0; q < kUpdDots; ++q) {
      const int j = j0 + q * kUpdBlock;
      dd[q] = j < nit ? dot[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kUpdDots; ++q) acc[1] -= dd[q];
  }
  {
    // a camera's item partials, summed by a group of kUpdLanes lanes: lane g takes items
    // g, g + kUpdLanes, ... in order, then a fixed tree over the group
    constexpr int kUpdLanes = kUpdBlock / kUpdCams;
    const int jc = int(threadIdx.x) / kUpdLanes, g = int(threadIdx.x) % kUpdLanes;
    const int sc = blockIdx.x * kUpdCams + jc;
    double ws[D];
#pragma unroll
    for (int i = 0; i < D; ++i) ws[i] = 0.0;
    if (sc < Ca) {
      const int i1 = item_off[sc + 1];
      for (int it = item_off[sc] + g; it < i1; it += kUpdLanes) {
#pragma unroll
        for (int i = 0; i < D; ++i) ws[i] += part[i * nslot + it];
      }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) ws[i] = group_sum<kUpdLanes>(ws[i]);
    if (g == 0) {
#pragma unroll
      for (int i = 0; i < D; ++i) s_items[jc][i] = ws[i];
    }
  }
  // thread 0 reads the state once for the whole workgroup
  int done0 = 0;
  double tol2 = 0.0, bb = 0.0, gprev = 0.0, aprev = 0.0;
  if (threadIdx.x == 0) {
    done0 = st->done;
    tol2 = st->tol2;
    bb = st->bb;
    gprev = st->gam[(k + 1) & 1];
    aprev = st->alp[(k + 1) & 1];
    s_go = !done0;
  }
  __syncthreads();
  if (!s_go) return;   // converged or broken down in an earlier iteration
  block_sum<double, 3>(acc, smem);
  if (threadIdx.x == 0) {
    const double gamma = acc[0], delta = acc[1], rho = acc[2];
    int go = !(rho <= tol2 * bb);
    int broke = 0;
    double alpha = 0.0, beta = 0.0;
    if (go) {
      beta = k == 0 ? 0.0 : gamma / gprev;
      const double den = k == 0 ? delta : delta - beta * gamma / aprev;
      alpha = gamma / den;
      if (!(den > 0.0) || !(gamma > 0.0) || !isfinite(alpha) || !isfinite(beta)) {
        broke = 1;
        go = 0;
      }
    }
    s_bcast[0] = alpha;
    s_bcast[1] = beta;
    s_go = go;
    if (blockIdx.x == 0) {
      st->rr = rho;
      st->matvecs += 1;
      if (go) {
        st->gam[k & 1] = gamma;
        st->alp[k & 1] = alpha;
        st->iter = k + 1;
      } else {
        st->breakdown = broke;
        st->done = 1;
      }
    }
  }
  __syncthreads();
  if (!s_go || !own) return;
  const double alpha = s_bcast[0], beta = s_bcast[1];
#pragma unroll
  for (int i = 0; i < D; ++i) wv[i] -= s_items[threadIdx.x][i];   // w = U* u - the partials
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double pi = uv[i] + beta * pv[i];
    const double si = wv[i] + beta * sv0[i];
    p[i * Ca + s] = pi;
    sv[i * Ca + s] = si;
    x[i * Ca + s] = xv[i] + alpha * pi;
    rv[i] -= alpha * si;
    r[i * Ca + s] = rv[i];
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) a += m[symd<D>(i, j)] * rv[j];
    uv[i] = a;
    u[i * Ca + s] = a;
    mvt[s].u[i] = T(a);
  }
  double ru = 0.0, uUu = 0.0, rr = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) a += double(us[symd<D>(i, j)]) * uv[j];
    Uu[i * Ca + s] = a;
    ru += rv[i] * uv[i];
    uUu += uv[i] * a;
    rr += rv[i] * rv[i];
  }
  tout[s] = ru;
  tout[Ca + s] = uUu;
  tout[2 * Ca + s] = rr;
}

// True residual of the PCG solution x at exit: the matvec passes are run once more on x
// itself (k_x_to_mv copies x into the matvec records and arms a state of its own), then
// k_true_residual forms S x = U* x - (the camera's item partials) and the float64 sums
// |b - S x|^2 and |b|^2, one workgroup in a fixed order.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
k_x_to_mv(int Ca, const double* __restrict__ x, MvRec<T, D>* __restrict__ mvt, PcgState* st) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) {
    st->done = 0;
    st->breakdown = 0;
  }
  if (s >= Ca) return;
#pragma unroll
  for (int i = 0; i < D; ++i) mvt[s].u[i] = T(x[i * Ca + s]);
}

template <typename T, int D>
__global__ void __launch_bounds__(1024)
k_true_residual(int Ca, const double* __restrict__ x, const double* __restrict__ b,
                const T* __restrict__ Ustar, const int* __restrict__ item_off, int nslot,
                const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double smem[2 * (1024 / kWave)];
  double acc[2] = {0.0, 0.0};   // |b - S x|^2, |b|^2
  for (int s = threadIdx.x; s < Ca; s += blockDim.x) {
    double xv[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xv[i] = x[i * Ca + s];
    const int i0 = item_off[s], i1 = item_off[s + 1];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) a += double(Ustar[symd<D>(i, j) * Ca + s]) * xv[j];
      for (int it = i0; it < i1; ++it) a -= part[i * nslot + it];
      const double bi = b[i * Ca + s];
      acc[0] += (bi - a) * (bi - a);
      acc[1] += bi * bi;
    }
  }
  block_sum<double, 2>(acc, smem);
  if (threadIdx.x == 0) {
    out[0] = acc[0];
    out[1] = acc[1];
  }
}

// Back-substitution dp = Vinv (b_p - sum_k W_k^T x_c) = hp - z, where hp = Vinv b_p comes from
// the damping setup and z = Vinv sum_k W_k^T x_c from the PCG point pass run on x (the camera
// step copied into the matvec records); with no solve camera (Ca = 0) dp = hp.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_backsub(int Pa, const double* __restrict__ hp, const P3<T>* __restrict__ zq, int use_z,
          double* __restrict__ dp) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= Pa) return;
  P3<T> z{T(0), T(0), T(0)};
  if (use_z) z = zq[r];
  dp[3 * r] = hp[3 * r] - double(z.x);
  dp[3 * r + 1] = hp[3 * r + 1] - double(z.y);
  dp[3 * r + 2] = hp[3 * r + 2] - double(z.z);
}

// ------------------------------------------------------------------ candidate
// Left SE(3) update of a (quaternion, centre) camera: q' = q(phi) (x) q, c' = c - R'^T V rho.
__global__ void __launch_bounds__(kBlock)
k_cam_candidate(int Ca, int Cf, int D, const int* __restrict__ cam_src,
                const double* __restrict__ x, const double* __restrict__ cams,
                const Cam<double>* __restrict__ camd_hat, double* __restrict__ cand_cams,
                Cam<double>* __restrict__ cand_tab) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= Ca + Cf) return;
  if (s >= Ca) {             // fixed camera: unchanged
    cand_tab[s] = camd_hat[s];
    return;
  }
  const int c = cam_src[s];
  const double rho[3] = {x[s], x[Ca + s], x[2 * Ca + s]};
  const double phi[3] = {x[3 * Ca + s], x[4 * Ca + s], x[5 * Ca + s]};
  const double t2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  const double th = sqrt(t2);
  double bco, cco, hco;
  if (th < 1e-2) {   // Taylor series where the closed forms lose digits
    bco = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
    cco = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0;
    hco = 0.5 - t2 / 48.0 + t2 * t2 / 3840.0;
  } else {
    bco = (1.0 - cos(th)) / t2;
    cco = (th - sin(th)) / (t2 * th);
    hco = sin(0.5 * th) / th;
  }
  const double cw = cos(0.5 * th);
  double qw = cams[7 * c], qx = cams[7 * c + 1], qy = cams[7 * c + 2], qz = cams[7 * c + 3];
  double n = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw /= n; qx /= n; qy /= n; qz /= n;
  const double aw = cw, ax = hco * phi[0], ay = hco * phi[1], az = hco * phi[2];
  double nw = aw * qw - ax * qx - ay * qy - az * qz;
  double nx = aw * qx + qw * ax + (ay * qz - az * qy);
  double ny = aw * qy + qw * ay + (az * qx - ax * qz);
  double nz = aw * qz + qw * az + (ax * qy - ay * qx);
  n = sqrt(nw * nw + nx * nx + ny * ny + nz * nz);
  nw /= n; nx /= n; ny /= n; nz /= n;
  Cam<double> d = camd_hat[s];
  d.R[0] = 1 - 2 * (ny * ny + nz * nz);
  d.R[1] = 2 * (nx * ny - nw * nz);
  d.R[2] = 2 * (nx * nz + nw * ny);
  d.R[3] = 2 * (nx * ny + nw * nz);
  d.R[4] = 1 - 2 * (nx * nx + nz * nz);
  d.R[5] = 2 * (ny * nz - nw * nx);
  d.R[6] = 2 * (nx * nz - nw * ny);
  d.R[7] = 2 * (ny * nz + nw * nx);
  d.R[8] = 1 - 2 * (nx * nx + ny * ny);
  double pr[3], ppr[3], vr[3];
  cross3(phi, rho, pr);
  cross3(phi, pr, ppr);
  for (int i = 0; i < 3; ++i) vr[i] = rho[i] + bco * pr[i] + cco * ppr[i];
  double rv[3];
  rot_tmul(d, vr, rv);
  d.c[0] = cams[7 * c + 4] - rv[0];
  d.c[1] = cams[7 * c + 5] - rv[1];
  d.c[2] = cams[7 * c + 6] - rv[2];
  if (D == 7) d.f += x[6 * Ca + s];   // additive focal update
  cand_tab[s] = d;
  cand_cams[7 * s] = nw;
  cand_cams[7 * s + 1] = nx;
  cand_cams[7 * s + 2] = ny;
  cand_cams[7 * s + 3] = nz;
  cand_cams[7 * s + 4] = d.c[0];
  cand_cams[7 * s + 5] = d.c[1];
  cand_cams[7 * s + 6] = d.c[2];
}

// Candidate evaluation over the same active observations (float64): the actual reduction
// sum_k (rho_k - rho'_k) / 2, summed per observation so that its rounding error scales with
// the changes rather than with the cost; the quadratic term of the model decrease
// sum w |J delta|^2 (Jacobian at the linearisation point); g_p.dp; the number of candidate
// depths <= min_depth; and the candidate cost itself.
// Points are tiled over the XCDs as in the linearisation (grid lin_point_blocks*), G lanes per
// point, so a wave reads its observations' streams in whole lines; every lane accumulates its
// own observations and the workgroup sums them in a fixed order. With LDS, B = 1024-thread
// workgroups first copy the candidate camera table into LDS (one 120-byte table fits; the
// current table stays in L2).
template <typename T, int G, int B, bool LDS>
__global__ void __launch_bounds__(B)
k_point_candidate(Model m, Compact<T> cp, int D, const Cam<double>* __restrict__ cand_tab,
                  const double* __restrict__ x, const double* __restrict__ dp,
                  const double* __restrict__ gp, const T* __restrict__ w,
                  double* __restrict__ Xcand, double* __restrict__ partials) {
  __shared__ double smem[5 * (B / kWave)];
  extern __shared__ double lds_cand[];   // LDS: the candidate camera table
  if constexpr (LDS) cand_tab = stage_cams<B>(cand_tab, cp.Ca + cp.Cf, lds_cand);
  const int per = gridDim.x / 8;
  const int xcd = blockIdx.x % 8, jw = blockIdx.x / 8;
  constexpr int tile = B / G;
  const int l = int(threadIdx.x) % G;
  const int Ca = cp.Ca;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // decrease, quad, g_p.dp, bad, cost'
  for (int t = 0; t < G; ++t) {
    const int r = xcd * per * B + (t * per + jw) * tile + int(threadIdx.x) / G;
    if (r >= cp.Pa) continue;
    const double X[3] = {cp.Xd[3 * r], cp.Xd[3 * r + 1], cp.Xd[3 * r + 2]};
    const double d[3] = {dp[3 * r], dp[3 * r + 1], dp[3 * r + 2]};
    const double Xn[3] = {X[0] + d[0], X[1] + d[1], X[2] + d[2]};
    if (l == 0) {
      Xcand[3 * r] = Xn[0];
      Xcand[3 * r + 1] = Xn[1];
      Xcand[3 * r + 2] = Xn[2];
      acc[2] += gp[3 * r] * d[0] + gp[3 * r + 1] * d[1] + gp[3 * r + 2] * d[2];
    }
    for (int j = cp.off[r] + l; j < cp.off[r + 1]; j += G) {
      const int s = cp.cam[j];
      const Cam<double> cm = cp.camd[s];
      double Xl[3], e[3], rho0, d1, d2;
      cam_frame(cm, X[0], X[1], X[2], Xl);
      residual(cm, Xl, cp.xy[j], cp.depth[j], m.lam_d, e);
      huber(e[0] * e[0] + e[1] * e[1] + e[2] * e[2], m.huber, rho0, d1, d2);
      const Cam<double> cn = cand_tab[s];
      double Xc[3];
      cam_frame(cn, Xn[0], Xn[1], Xn[2], Xc);
      if (!(Xc[2] > m.min_depth)) {
        acc[3] += 1.0;
      } else {
        double e2[3], rho;
        residual(cn, Xc, cp.xy[j], cp.depth[j], m.lam_d, e2);
        huber(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2], m.huber, rho, d1, d2);
        acc[0] += 0.5 * (rho0 - rho);
        acc[4] += 0.5 * rho;
      }
      // model term at the linearisation point
      double v[3], tv[3];
      rot_mul(cm, d, v);
      if (s < Ca) {
        const double w3[3] = {x[3 * Ca + s], x[4 * Ca + s], x[5 * Ca + s]};
        double o3[3];
        cross3(w3, Xl, o3);
        v[0] += x[s] + o3[0];
        v[1] += x[Ca + s] + o3[1];
        v[2] += x[2 * Ca + s] + o3[2];
      }
      AMat<double, false> A;
      A.set(cm.f, m.lam_d, Xl);
      A.apply(v, tv);
      if (D == 7 && s < Ca) {   // focal column times the camera's focal step
        const double uf = x[6 * Ca + s] / Xl[2];
        tv[0] += Xl[0] * uf;
        tv[1] += Xl[1] * uf;
      }
      acc[1] += double(w[j]) * (tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2]);
    }
  }
  block_sum<double, 5>(acc, smem);
  if (threadIdx.x == 0) {
    const int blk = xcd * per + jw;
#pragma unroll
    for (int i = 0; i < 5; ++i) partials[5 * blk + i] = acc[i];
  }
}

__global__ void __launch_bounds__(1024)
k_reduce_partials(int nb, int K, const double* __restrict__ partials, unsigned max_mask,
                  int ncu, const double* __restrict__ gc, const double* __restrict__ x,
                  double* __restrict__ out) {
  constexpr int KM = 8;
  __shared__ double smem[KM * (1024 / kWave)];
  double acc[KM];
  for (int k = 0; k < KM; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    for (int k = 0; k < K; ++k) {
      const double v = partials[K * b + k];
      acc[k] = ((max_mask >> k) & 1u) ? fmax(acc[k], v) : acc[k] + v;
    }
  }
  unsigned mask = max_mask;
  int nout = K;
  if (gc) {
    // gc . x over the ncu camera unknowns (D per camera, SoA), and max |gc|
    for (int e = threadIdx.x; e < ncu; e += blockDim.x) {
      acc[K] += gc[e] * x[e];
      acc[K + 1] = fmax(acc[K + 1], fabs(gc[e]));
    }
    mask |= 1u << (K + 1);
    nout = K + 2;
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int k = 0; k < KM; ++k) acc[k] = ((mask >> k) & 1u) ? wave_max(acc[k]) : wave_sum(acc[k]);
  if (lane == 0)
    for (int k = 0; k < KM; ++k) smem[KM * wid + k] = acc[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < nout; ++k) {
      double a = smem[k];
      for (int w = 1; w < int(blockDim.x) / kWave; ++w)
        a = ((mask >> k) & 1u) ? fmax(a, smem[KM * w + k]) : a + smem[KM * w + k];
      out[k] = a;
    }
  }
}

__global__ void __launch_bounds__(kBlock)
k_scatter(int Pa, int Ca, const int* __restrict__ pt_src, const double* __restrict__ Xcand,
          const int* __restrict__ cam_src, const double* __restrict__ cand_cams,
          const Cam<double>* __restrict__ cand_tab, double* __restrict__ pts,
          double* __restrict__ cams, double* __restrict__ intr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < Pa) {
    const int p = pt_src[i];
    pts[3 * p] = Xcand[3 * i];
    pts[3 * p + 1] = Xcand[3 * i + 1];
    pts[3 * p + 2] = Xcand[3 * i + 2];
  }
  if (i < Ca) {
    const int c = cam_src[i];
    for (int k = 0; k < 7; ++k) cams[7 * c + k] = cand_cams[7 * i + k];
    if (intr) intr[3 * c] = cand_tab[i].f;   // refined focal length
  }
}

// ------------------------------------------------------------------ adjoint
// Tangent mapping of camera gradients: dL/drho = -R dL/dc, dL/dphi = (dq/dphi)^T dL/dq with
// dq/dphi = 1/2 [-q_v^T ; q_w I - [q_v]x]. Output SoA like every camera vector.
__global__ void __launch_bounds__(kBlock)
k_adjoint_rhs(int Ca, int Pa, const int* __restrict__ cam_src, const double* __restrict__ cams,
              const double* __restrict__ grad_cams, const int* __restrict__ pt_src,
              const int* __restrict__ pt_user, const double* __restrict__ grad_pts,
              double* __restrict__ rhs_c, double* __restrict__ rhs_p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < Ca) {
    const int c = cam_src[i];
    double qw = cams[7 * c], qx = cams[7 * c + 1], qy = cams[7 * c + 2], qz = cams[7 * c + 3];
    const double n = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= n; qx /= n; qy /= n; qz /= n;
    Cam<double> d;
    d.R[0] = 1 - 2 * (qy * qy + qz * qz);
    d.R[1] = 2 * (qx * qy - qw * qz);
    d.R[2] = 2 * (qx * qz + qw * qy);
    d.R[3] = 2 * (qx * qy + qw * qz);
    d.R[4] = 1 - 2 * (qx * qx + qz * qz);
    d.R[5] = 2 * (qy * qz - qw * qx);
    d.R[6] = 2 * (qx * qz - qw * qy);
    d.R[7] = 2 * (qy * qz + qw * qx);
    d.R[8] = 1 - 2 * (qx * qx + qy * qy);
    const double* g = grad_cams + 7 * c;
    const double gcn[3] = {g[4], g[5], g[6]};
    double rg[3];
    rot_mul(d, gcn, rg);
    const double qv[3] = {qx, qy, qz}, gv[3] = {g[1], g[2], g[3]};
    double cx[3];
    cross3(qv, gv, cx);
    for (int k = 0; k < 3; ++k) {
      rhs_c[k * Ca + i] = -rg[k];
      rhs_c[(3 + k) * Ca + i] = 0.5 * (-g[0] * qv[k] + qw * gv[k] + cx[k]);
    }
  }
  if (i < Pa) {
    const int u = pt_user[pt_src[i]];
    rhs_p[3 * i] = grad_pts[3 * u];
    rhs_p[3 * i + 1] = grad_pts[3 * u + 1];
    rhs_p[3 * i + 2] = grad_pts[3 * u + 2];
  }
}

// Per observation: t = J v, u = M t = w (I - eh eh^T) t; dL/dx = u[0:2],
// dL/dd_hat = -u[2] lam_d m / d_hat^2.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adjoint_obs(Model m, Compact<T> cp, ObsMetric<T> om, const double* __restrict__ x,
              const double* __restrict__ dp, const int* __restrict__ orig,
              float* __restrict__ gxy, float* __restrict__ gdepth) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= cp.Pa) return;
  const int Ca = cp.Ca;
  const double X0 = cp.Xd[3 * r], X1 = cp.Xd[3 * r + 1], X2 = cp.Xd[3 * r + 2];
  const double vp[3] = {dp[3 * r], dp[3 * r + 1], dp[3 * r + 2]};
  for (int j = cp.off[r]; j < cp.off[r + 1]; ++j) {
    const int s = cp.cam[j];
    const Cam<double> cm = cp.camd[s];
    double Xc[3], d[3], t[3];
    cam_frame(cm, X0, X1, X2, Xc);
    rot_mul(cm, vp, d);
    if (s < Ca) {
      const double w3[3] = {x[3 * Ca + s], x[4 * Ca + s], x[5 * Ca + s]};
      double o3[3];
      cross3(w3, Xc, o3);
      d[0] += x[s] + o3[0];
      d[1] += x[Ca + s] + o3[1];
      d[2] += x[2 * Ca + s] + o3[2];
    }
    AMat<double, true> A;
    A.set(cm.f, m.lam_d, Xc);
    const double eh[3] = {double(om.eh[3 * j]), double(om.eh[3 * j + 1]),
                          double(om.eh[3 * j + 2])};
    A.project(eh);
    A.apply(d, t);
    const double w = double(om.w[j]);
    const int o = orig[j];
    gxy[2 * o] = float(w * t[0]);
    gxy[2 * o + 1] = float(w * t[1]);
    const float dh = cp.depth[j];
    const double dinv = dh > 0.0f ? 1.0 / double(dh) : 0.0;
    gdepth[o] = float(-w * t[2] * m.lam_d * dinv * dinv);
  }
}

// ------------------------------------------------------------------ explicit reduced system
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_pair_counts(Compact<T> cp, int64_t* __restrict__ cnt, int* __restrict__ pm_rank) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= cp.Pa) return;
  int64_t m = 0;
  for (int j = cp.off[r]; j < cp.off[r + 1]; ++j) {
    pm_rank[j] = r;
    m += cp.cam[j] < cp.Ca ? 1 : 0;
  }
  cnt[r] = m * (m - 1);
}

// G lanes per point; lane l writes the contributions whose first observation is its a-th
// solve observation (a = l, l + G, ...), in the order (a, then b) of the point's list.
template <typename T, int G>
__global__ void __launch_bounds__(kBlock)
k_pair_keys(Compact<T> cp, const int64_t* __restrict__ coff, uint32_t* __restrict__ key,
            uint64_t* __restrict__ val) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = t / G, l = t % G;
  if (r >= cp.Pa) return;
  const uint32_t Ca = uint32_t(cp.Ca);
  const int b0 = cp.off[r], b1 = cp.off[r + 1];
  int64_t m = 0;
  for (int j = b0; j < b1; ++j) m += cp.cam[j] < cp.Ca ? 1 : 0;
  int ia = 0;   // index of a among the solve observations
  for (int a = b0; a < b1; ++a) {
    const int sa = cp.cam[a];
    if (sa >= cp.Ca) continue;
    if (ia % G == l) {
      int64_t c = coff[r] + int64_t(ia) * (m - 1);
      for (int b = b0; b < b1; ++b) {
        const int sb = cp.cam[b];
        if (b == a || sb >= cp.Ca) continue;
        key[c] = uint32_t(sa) * Ca + uint32_t(sb);
        val[c] = (uint64_t(uint32_t(a)) << 32) | uint64_t(uint32_t(b));
        ++c;
      }
    }
    ++ia;
  }
}

__global__ void __launch_bounds__(kBlock)
k_run_flags(int64_t n, const uint32_t* __restrict__ key, int64_t* __restrict__ flag) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= n) return;
  flag[c] = (c == 0 || key[c] != key[c - 1]) ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock)
k_block_list(int64_t n, const uint32_t* __restrict__ key, const int64_t* __restrict__ flag,
             const int64_t* __restrict__ bidx, uint32_t* __restrict__ bkey,
             int64_t* __restrict__ bstart) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= n || !flag[c]) return;
  bkey[bidx[c]] = key[c];
  bstart[bidx[c]] = c;
}

__global__ void __launch_bounds__(kBlock)
k_block_rows(int Ca, int64_t nb, const uint32_t* __restrict__ bkey, int64_t* __restrict__ row_ptr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > Ca) return;
  // first block whose row is >= i
  const uint32_t target = uint32_t(i) * uint32_t(Ca);
  int64_t lo = 0, hi = nb;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (bkey[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  row_ptr[i] = lo;
}

// W = J_c^T w J_p (D x 3) of one observation from its (X_c, w) and its camera.
template <typename T, int D>
__device__ __forceinline__ void w_block(const Cam<T>& cm, T lam_d, const V4<T>& xw,
                                        T W[D][3]) {
  const T Xc[3] = {xw.x, xw.y, xw.z};
  AMat<T, false> A;
  A.set(cm.f, lam_d, Xc);
#pragma unroll
  for (int p = 0; p < D; ++p) W[p][0] = W[p][1] = W[p][2] = T(0);
#pragma unroll
  for (int row = 0; row < 3; ++row) {
    T a[3], jc[D], jp[3];
    A.row(row, a);
    jc[0] = a[0];
    jc[1] = a[1];
    jc[2] = a[2];
    cross3(Xc, a, jc + 3);
    if constexpr (D == 7) jc[6] = row < 2 ? Xc[row] / Xc[2] : T(0);
    rot_tmul(cm, a, jp);
#pragma unroll
    for (int p = 0; p < D; ++p) {
      const T wj = xw.w * jc[p];
      W[p][0] += wj * jp[0];
      W[p][1] += wj * jp[1];
      W[p][2] += wj * jp[2];
    }
  }
}

// One wave per off-diagonal block (i, j): lanes take its contributions in turn, the wave sums
// them in a fixed shuffle order.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
k_schur_blocks(Model m, Compact<T> cp, ObsMetric<T> om, const T* __restrict__ Vinv,
               const int* __restrict__ pm_rank, int64_t nb, const uint32_t* __restrict__ bkey,
               const int64_t* __restrict__ bstart, const uint64_t* __restrict__ sval,
               T* __restrict__ sblk) {
  const int64_t b = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (b >= nb) return;   // whole waves leave together
  const uint32_t Ca = uint32_t(cp.Ca);
  const int ci = int(bkey[b] / Ca), cj = int(bkey[b] % Ca);
  const Cam<T> cmi = cp.camt[ci], cmj = cp.camt[cj];
  const T lam_d = T(m.lam_d);
  T acc[D * D];
#pragma unroll
  for (int q = 0; q < D * D; ++q) acc[q] = T(0);
  for (int64_t c = bstart[b] + lane; c < bstart[b + 1]; c += kWave) {
    const uint64_t v = sval[c];
    const int k = int(v >> 32), l = int(v & 0xffffffffu);
    const int r = pm_rank[k];
    T Wk[D][3], Wl[D][3];
    w_block<T, D>(cmi, lam_d, om.pm_xcw[k], Wk);
    w_block<T, D>(cmj, lam_d, om.pm_xcw[l], Wl);
    T vi[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) vi[q] = Vinv[6 * r + q];
    T Y[D][3];
#pragma unroll
    for (int p = 0; p < D; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        Y[p][q] = Wk[p][0] * vi[sym3(0, q)] + Wk[p][1] * vi[sym3(1, q)] +
                  Wk[p][2] * vi[sym3(2, q)];
#pragma unroll
    for (int p = 0; p < D; ++p)
#pragma unroll
      for (int q = 0; q < D; ++q)
        acc[p * D + q] += Y[p][0] * Wl[q][0] + Y[p][1] * Wl[q][1] + Y[p][2] * Wl[q][2];
  }
#pragma unroll
  for (int q = 0; q < D * D; ++q) acc[q] = wave_sum(acc[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < D * D; ++q) sblk[b * (D * D) + q] = -acc[q];
  }
}

// One wave per block row of S: w_i = S_cc u_i + sum over its off-diagonal blocks S_b u_j.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
k_schur_spmv(int Ca, const int64_t* __restrict__ row_ptr, const uint32_t* __restrict__ bkey,
             const T* __restrict__ sblk, const double* __restrict__ Scc,
             const double* __restrict__ u, const double* __restrict__ Uu, int nslot,
             double* __restrict__ part, const PcgState* __restrict__ st) {
  if (st->done) return;
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (i >= Ca) return;
  T y[D];
#pragma unroll
  for (int p = 0; p < D; ++p) y[p] = T(0);
  for (int64_t b = row_ptr[i] + lane; b < row_ptr[i + 1]; b += kWave) {
    const int j = int(bkey[b] % uint32_t(Ca));
    T uj[D];
#pragma unroll
    for (int q = 0; q < D; ++q) uj[q] = T(u[q * Ca + j]);
    const T* S = sblk + b * (D * D);
#pragma unroll
    for (int p = 0; p < D; ++p) {
      T a = T(0);
#pragma unroll
      for (int q = 0; q < D; ++q) a += S[p * D + q] * uj[q];
      y[p] += a;
    }
  }
#pragma unroll
  for (int p = 0; p < D; ++p) y[p] = wave_sum(y[p]);
  if (lane != 0) return;
  double ui[D];
#pragma unroll
  for (int q = 0; q < D; ++q) ui[q] = u[q * Ca + i];
  double pd = 0.0;
#pragma unroll
  for (int p = 0; p < D; ++p) {
    double w = double(y[p]);
#pragma unroll
    for (int q = 0; q < D; ++q) w += Scc[symd<D>(p, q) * Ca + i] * ui[q];
    const double pt = Uu[p * Ca + i] - w;
    part[p * nslot + i] = pt;
    pd += ui[p] * pt;
  }
  part[D * nslot + i] = pd;
}

// ------------------------------------------------------------------ global positioning
// Unit world ray of an observation: v = R^T a / |a| with a = K^-1 [x, y, 1]; returns |a|.
__device__ __forceinline__ double gp_ray(const Cam<double>& cm, float2 xy, double v[3]) {
  const double a[3] = {(double(xy.x) - cm.cx) / cm.f, (double(xy.y) - cm.cy) / cm.f, 1.0};
  const double na = sqrt(a[0] * a[0] + a[1] * a[1] + 1.0);
  double t[3];
  rot_tmul(cm, a, t);
  v[0] = t[0] / na;
  v[1] = t[1] / na;
  v[2] = t[2] / na;
  return na;
}

__global__ void __launch_bounds__(kBlock)
k_gp_validate(int64_t N, const float2* __restrict__ xy, const float* __restrict__ depth,
              const int* __restrict__ inv_cm, uint8_t* __restrict__ vrow,
              uint8_t* __restrict__ vrow_cm) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const float2 p = xy[k];
  const uint8_t rows = (isfinite(p.x) && isfinite(p.y)) ? (depth[k] > 0.0f ? 3 : 2) : 0;
  vrow[k] = rows;
  vrow_cm[inv_cm[k]] = rows;
}

__global__ void __launch_bounds__(kBlock)
k_gp_init_scales(int64_t N, const int* __restrict__ pm_cam, const int* __restrict__ pm_pt,
                 const int* __restrict__ pm_orig, const float2* __restrict__ xy,
                 const float* __restrict__ depth, const double* __restrict__ pts,
                 const Cam<double>* __restrict__ camd, double* __restrict__ scales) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const Cam<double> cm = camd[pm_cam[k]];
  const int p = pm_pt[k];
  double v[3];
  const double na = gp_ray(cm, xy[k], v);
  const float dh = depth[k];
  double sc;
  if (dh > 0.0f) {
    sc = 1.0 / (double(dh) * na);
  } else {
    const double d0 = pts[3 * p] - cm.c[0], d1 = pts[3 * p + 1] - cm.c[1];
    const double d2 = pts[3 * p + 2] - cm.c[2];
    sc = 1.0 / fmax(sqrt(d0 * d0 + d1 * d1 + d2 * d2), 1e-12);
  }
  scales[pm_orig[k]] = sc;
}

// Residual of one compact observation at the current estimate (float64).
struct GpObs {
  double v[3], d[3], u[3], s;
  bool pinned;
};
__device__ __forceinline__ GpObs gp_obs(const Cam<double>& cm, float2 xy, float dh,
                                        const double X[3], double s_free) {
  GpObs o;
  const double na = gp_ray(cm, xy, o.v);
  o.pinned = dh > 0.0f;
  o.s = o.pinned ? 1.0 / (double(dh) * na) : s_free;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o.d[i] = X[i] - cm.c[i];
    o.u[i] = o.v[i] - o.s * o.d[i];
  }
  return o;
}

template <typename T, int G, int B, bool LDS>
__global__ void __launch_bounds__(B)
k_gp_lin(Compact<T> cp, const int* __restrict__ orig, const double* __restrict__ scales,
         double delta, GpLin<T>* __restrict__ lin_pm, GpLin<T>* __restrict__ lin_cm,
         double* __restrict__ gX, double* __restrict__ partials) {
  __shared__ double smem[3 * (B / kWave)];
  extern __shared__ double lds_cam[];   // LDS: the compact camera table
  const Cam<double>* camtab = cp.camd;
  if constexpr (LDS) camtab = stage_cams<B>(cp.camd, cp.Ca + cp.Cf, lds_cam);
  const int per = gridDim.x / 8;
  const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
  constexpr int tile = B / G;
  const int l = int(threadIdx.x) % G;
  double acc[3] = {0.0, 0.0, 0.0};   // cost, sum |u|^2, max |g|
  for (int t = 0; t < G; ++t) {
    const int r = blk * B + t * tile + int(threadIdx.x) / G;
    const bool live = r < cp.Pa;
    double g[3] = {0.0, 0.0, 0.0};
    if (live) {
      const double X[3] = {cp.Xd[3 * r], cp.Xd[3 * r + 1], cp.Xd[3 * r + 2]};
      for (int j = cp.off[r] + l; j < cp.off[r + 1]; j += G) {
        const Cam<double> cm = camtab[cp.cam[j]];
        const float dh = cp.depth[j];
        const GpObs o = gp_obs(cm, cp.xy[j], dh, X, dh > 0.0f ? 0.0 : scales[orig[j]]);
        const double e2 = o.u[0] * o.u[0] + o.u[1] * o.u[1] + o.u[2] * o.u[2];
        double rho, w, d2;
        huber(e2, delta, rho, w, d2);
        acc[0] += 0.5 * rho;
        acc[1] += e2;
        const double ws = w * o.s;
        g[0] -= ws * o.u[0];
        g[1] -= ws * o.u[1];
        g[2] -= ws * o.u[2];
        if (!o.pinned) {   // g_s = -w d.u
          const double gs = -w * (o.d[0] * o.u[0] + o.d[1] * o.u[1] + o.d[2] * o.u[2]);
          acc[2] = fmax(acc[2], fabs(gs));
        }
        GpLin<T> rec;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          rec.d[i] = T(o.d[i]);
          rec.u[i] = T(o.u[i]);
        }
        rec.s = T(o.pinned ? -o.s : o.s);
        rec.w = T(w);
        lin_pm[j] = rec;
        const int ic = cp.pm_cm[j];
        if (ic >= 0) lin_cm[ic] = rec;
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = group_sum<G>(g[i]);
    if (live && l == 0) {
      gX[3 * r] = g[0];
      gX[3 * r + 1] = g[1];
      gX[3 * r + 2] = g[2];
      acc[2] = fmax(acc[2], fmax(fabs(g[0]), fmax(fabs(g[1]), fabs(g[2]))));
    }
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  acc[0] = wave_sum(acc[0]);
  acc[1] = wave_sum(acc[1]);
  acc[2] = wave_max(acc[2]);
  if (lane == 0) {
    smem[3 * wid] = acc[0];
    smem[3 * wid + 1] = acc[1];
    smem[3 * wid + 2] = acc[2];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int w = 0; w < int(blockDim.x) / kWave; ++w) {
      a0 += smem[3 * w];
      a1 += smem[3 * w + 1];
      a2 = fmax(a2, smem[3 * w + 2]);
    }
    partials[3 * blk] = a0;
    partials[3 * blk + 1] = a1;
    partials[3 * blk + 2] = a2;
  }
}

// Scale elimination of one linearised observation: a0 = w s^2, the coupling vector e (zero
// when pinned), and q = w s (u + d g_s / h*) (the observation's share of the reduced RHS).
template <typename T>
__device__ __forceinline__ void gp_reduce(const GpLin<T>& L, double lam, double dmin,
                                          double dmax, double e[3], double& a0, double q[3]) {
  const double w = double(L.w);
  const bool pinned = L.s < T(0);
  const double s = pinned ? -double(L.s) : double(L.s);
  const double d[3] = {double(L.d[0]), double(L.d[1]), double(L.d[2])};
  const double u[3] = {double(L.u[0]), double(L.u[1]), double(L.u[2])};
  a0 = w * s * s;
  double f = 0.0, ce = 0.0;
  if (!pinned) {
    const double h = w * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double hs = h + lam * fmin(fmax(h, dmin), dmax);
    const double gs = -w * (d[0] * u[0] + d[1] * u[1] + d[2] * u[2]);
    f = gs / hs;
    ce = w * s / sqrt(hs);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    e[i] = ce * d[i];
    q[i] = w * s * (u[i] + d[i] * f);
  }
}

// A x = a0 x - e (e . x)
template <typename T>
__device__ __forceinline__ void gp_apply(const V4<T>& a, const T x[3], T y[3]) {
  const T ex = a.x * x[0] + a.y * x[1] + a.z * x[2];
  y[0] = a.w * x[0] - a.x * ex;
  y[1] = a.w * x[1] - a.y * ex;
  y[2] = a.w * x[2] - a.z * ex;
}

template <typename T, int G>
__global__ void __launch_bounds__(kBlock)
k_gp_point_setup(Compact<T> cp, double lam, double dmin, double dmax,
                 const GpLin<T>* __restrict__ lin_pm, V4<T>* __restrict__ a_pm,
                 V4<T>* __restrict__ a_cm, T* __restrict__ Vinv, double* __restrict__ hp,
                 PtRec<T>* __restrict__ prec, int* __restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = t / G;
  const int l = t % G;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};   // sum A (6, upper triangle), sum a0
  double q[3] = {0, 0, 0};
  if (r < cp.Pa) {
    for (int j = cp.off[r] + l; j < cp.off[r + 1]; j += G) {
      double e[3], a0, qk[3];
      gp_reduce(lin_pm[j], lam, dmin, dmax, e, a0, qk);
      V4<T> rec;
      rec.x = T(e[0]);
      rec.y = T(e[1]);
      rec.z = T(e[2]);
      rec.w = T(a0);
      a_pm[j] = rec;
      const int ic = cp.pm_cm[j];
      if (ic >= 0) a_cm[ic] = rec;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
#pragma unroll
        for (int k = p; k < 3; ++k) v[sym3(p, k)] += (p == k ? a0 : 0.0) - e[p] * e[k];
        q[p] += qk[p];
      }
      v[6] += a0;
    }
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) v[i] = group_sum<G>(v[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) q[i] = group_sum<G>(q[i]);
  if (r >= cp.Pa || l != 0) return;
  const double dmp = lam * fmin(fmax(v[6], dmin), dmax);
  const double v00 = v[0] + dmp, v01 = v[1], v02 = v[2];
  const double v11 = v[3] + dmp, v12 = v[4], v22 = v[5] + dmp;
  const double c00 = v11 * v22 - v12 * v12;
  const double c01 = v02 * v12 - v01 * v22;
  const double c02 = v01 * v12 - v02 * v11;
  const double c11 = v00 * v22 - v02 * v02;
  const double c12 = v01 * v02 - v00 * v12;
  const double c22 = v00 * v11 - v01 * v01;
  const double det = v00 * c00 + v01 * c01 + v02 * c02;
  double inv[6] = {0, 0, 0, 0, 0, 0};
  if (det > 0.0 && isfinite(det)) {
    const double id = 1.0 / det;
    inv[0] = c00 * id; inv[1] = c01 * id; inv[2] = c02 * id;
    inv[3] = c11 * id; inv[4] = c12 * id; inv[5] = c22 * id;
  } else {
    *bad = 1;
  }
  PtRec<T> rec;
  rec.hp[0] = inv[0] * q[0] + inv[1] * q[1] + inv[2] * q[2];
  rec.hp[1] = inv[1] * q[0] + inv[3] * q[1] + inv[4] * q[2];
  rec.hp[2] = inv[2] * q[0] + inv[4] * q[1] + inv[5] * q[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) hp[3 * r + i] = rec.hp[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    rec.vinv[i] = T(inv[i]);
    Vinv[6 * r + i] = T(inv[i]);
  }
  prec[r] = rec;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_gp_cam_assemble(Compact<T> cp, double lam, double dmin, double dmax,
                  const GpLin<T>* __restrict__ lin_cm, const V4<T>* __restrict__ a_cm,
                  const PtRec<T>* __restrict__ prec, T* __restrict__ Ustar,
                  double* __restrict__ gc, double* __restrict__ b, double* __restrict__ Minv) {
  constexpr int K = 6 + 1 + 6 + 3 + 3 + 3;   // U, sum a0, sum A Vinv A, g_c, r_c, sum A hp
  __shared__ double smem[K * (kBlock / kWave)];
  const int s = blockIdx.x;
  const int Ca = cp.Ca;
  double acc[K];
#pragma unroll
  for (int i = 0; i < K; ++i) acc[i] = 0.0;
  for (int i = cp.cm_off[s] + threadIdx.x; i < cp.cm_off[s + 1]; i += blockDim.x) {
    const GpLin<T> L = lin_cm[i];
    const V4<T> ar = a_cm[i];
    const PtRec<T> pr = prec[cp.cm_pt[i]];
    double e[3], a0, q[3];
    gp_reduce(L, lam, dmin, dmax, e, a0, q);
    const double w = double(L.w);
    const double sc = L.s < T(0) ? -double(L.s) : double(L.s);
    // A (float64 from the record's own values) and A Vinv A
    double Am[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        Am[p][k] = (p == k ? double(ar.w) : 0.0) -
                   double(p == 0 ? ar.x : p == 1 ? ar.y : ar.z) *
                       double(k == 0 ? ar.x : k == 1 ? ar.y : ar.z);
    double AV[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        AV[p][k] = Am[p][0] * double(pr.vinv[sym3(0, k)]) +
                   Am[p][1] * double(pr.vinv[sym3(1, k)]) +
                   Am[p][2] * double(pr.vinv[sym3(2, k)]);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int k = p; k < 3; ++k) {
        acc[sym3(p, k)] += Am[p][k];
        acc[7 + sym3(p, k)] += AV[p][0] * Am[0][k] + AV[p][1] * Am[1][k] + AV[p][2] * Am[2][k];
      }
      acc[13 + p] += w * sc * double(L.u[p]);
      acc[16 + p] -= q[p];
      acc[19 + p] += Am[p][0] * pr.hp[0] + Am[p][1] * pr.hp[1] + Am[p][2] * pr.hp[2];
    }
    acc[6] += a0;
  }
  block_sum<double, K>(acc, smem);
  if (threadIdx.x != 0) return;
  const double dmp = lam * fmin(fmax(acc[6], dmin), dmax);
  double Us[6], Sc[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) Us[q] = acc[q];
  Us[sym3(0, 0)] += dmp;
  Us[sym3(1, 1)] += dmp;
  Us[sym3(2, 2)] += dmp;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    Ustar[q * Ca + s] = T(Us[q]);
    Sc[q] = Us[q] - acc[7 + q];
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    gc[p * Ca + s] = acc[13 + p];
    b[p * Ca + s] = acc[16 + p] + acc[19 + p];
  }
  double inv[6];
  if (!spd_inverse<3>(Sc, inv)) {
#pragma unroll
    for (int q = 0; q < 6; ++q) inv[q] = 0.0;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const double d = Us[sym3(p, p)];
      inv[sym3(p, p)] = d > 0.0 ? 1.0 / d : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) Minv[q * Ca + s] = inv[q];
}

// Point pass: y_p = sum_k A_k u_c, zz_p = V*^-1 y_p stored at the camera-major position of
// each observation of p in a solve camera. XCD-contiguous point ranges as in BA.
template <typename T, int G>
__global__ void __launch_bounds__(kBlock)
k_gp_schur_point(Compact<T> cp, const V4<T>* __restrict__ a_pm,
                 const GpMv<T>* __restrict__ mvt, const T* __restrict__ Vinv,
                 P3<T>* __restrict__ zq_cm, const PcgState* __restrict__ st) {
  if (st->done) return;
  const int per = gridDim.x / 8;
  const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const int t = blk * blockDim.x + threadIdx.x;
  const int r = t / G;
  const int l = t % G;
  T y[3] = {T(0), T(0), T(0)};
  int b = 0, e = 0;
  const bool live = r < cp.Pa;
  if (live) {
    b = cp.off[r];
    e = cp.off[r + 1];
    for (int j = b + l; j < e; j += G) {
      const int s = cp.cam[j];
      if (s >= cp.Ca) continue;
      const GpMv<T> mc = mvt[s];
      T o[3];
      gp_apply(a_pm[j], mc.u, o);
      y[0] += o[0];
      y[1] += o[1];
      y[2] += o[2];
    }
  }
  y[0] = group_sum<G>(y[0]);
  y[1] = group_sum<G>(y[1]);
  y[2] = group_sum<G>(y[2]);
  if (!live) return;
  T vi[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) vi[q] = Vinv[6 * r + q];
  P3<T> z;
  z.x = vi[0] * y[0] + vi[1] * y[1] + vi[2] * y[2];
  z.y = vi[1] * y[0] + vi[3] * y[1] + vi[4] * y[2];
  z.z = vi[2] * y[0] + vi[4] * y[1] + vi[5] * y[2];
  for (int j = b + l; j < e; j += G) {
    const int pos = cp.pm_cm[j];
    if (pos >= 0) zq_cm[pos] = z;
  }
}

// The same with the camera records in LDS, over a grid-stride walk of point tiles (XCD x owns
// the x-th eighth of the point ranks, as in the bundle-adjustment point pass); the next
// tile's first-observation data (slot, A_k, camera-major position) are loaded before the
// current tile is worked on.
template <typename T>
struct GpPtLoad {
  int b, e, s0, pos0;
  V4<T> a0;
};

template <typename T, int G>
__device__ __forceinline__ void gp_pt_load_first(const Compact<T>& cp,
                                                 const V4<T>* __restrict__ a_pm, int l,
                                                 GpPtLoad<T>& p) {
  p.s0 = cp.Ca;
  p.pos0 = -1;
  p.a0.x = p.a0.y = p.a0.z = p.a0.w = T(0);
  if (p.b + l < p.e) {
    p.s0 = cp.cam[p.b + l];
    p.a0 = a_pm[p.b + l];
    p.pos0 = cp.pm_cm[p.b + l];
  }
}

template <typename T, int G>
__global__ void __launch_bounds__(kPtLdsBlock)
k_gp_schur_point_lds(Compact<T> cp, const V4<T>* __restrict__ a_pm,
                     const GpMv<T>* __restrict__ mvt, const T* __restrict__ Vinv,
                     P3<T>* __restrict__ zq_cm, const PcgState* __restrict__ st, int ppx) {
  extern __shared__ uint4 lds_tab[];   // cp.Ca records
  if (st->done) return;
  const int per = gridDim.x / 8;
  const int xcd = blockIdx.x % 8;
  const int jw = blockIdx.x / 8;
  const int lo = xcd * ppx;
  const int hi = min(cp.Pa, lo + ppx);
  constexpr int tile = kPtLdsBlock / G;
  const int step = per * tile;
  const int l = int(threadIdx.x) % G;
  int r = lo + jw * tile + int(threadIdx.x) / G;
  GpPtLoad<T> cur;
  cur.b = r < hi ? cp.off[r] : 0;
  cur.e = r < hi ? cp.off[r + 1] : 0;
  gp_pt_load_first<T, G>(cp, a_pm, l, cur);
  int bn = 0, en = 0;
  if (r + step < hi) {
    bn = cp.off[r + step];
    en = cp.off[r + step + 1];
  }
  const int nchunk = cp.Ca * int(sizeof(GpMv<T>) / sizeof(uint4));
  const uint4* src = reinterpret_cast<const uint4*>(mvt);
  for (int i = threadIdx.x; i < nchunk; i += kPtLdsBlock) lds_tab[i] = src[i];
  __syncthreads();
  const GpMv<T>* tab = reinterpret_cast<const GpMv<T>*>(lds_tab);
  for (int base = lo + jw * tile; base < hi; base += step, r += step) {
    GpPtLoad<T> nxt;
    nxt.b = bn;
    nxt.e = en;
    gp_pt_load_first<T, G>(cp, a_pm, l, nxt);
    bn = en = 0;
    if (r + 2 * step < hi) {
      bn = cp.off[r + 2 * step];
      en = cp.off[r + 2 * step + 1];
    }
    const bool live = r < hi;
    T y[3] = {T(0), T(0), T(0)};
    T vi[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if (live) {
#pragma unroll
      for (int q = 0; q < 6; ++q) vi[q] = Vinv[6 * r + q];
      auto obs = [&](int sj, const V4<T>& a) {
        if (sj >= cp.Ca) return;
        T o[3];
        gp_apply(a, tab[sj].u, o);
        y[0] += o[0];
        y[1] += o[1];
        y[2] += o[2];
      };
      int j = cur.b + l;
      if (j < cur.e) {
        obs(cur.s0, cur.a0);
        for (j += G; j < cur.e; j += G) obs(cp.cam[j], a_pm[j]);
      }
    }
    y[0] = group_sum<G>(y[0]);
    y[1] = group_sum<G>(y[1]);
    y[2] = group_sum<G>(y[2]);
    if (live) {
      P3<T> z;
      z.x = vi[0] * y[0] + vi[1] * y[1] + vi[2] * y[2];
      z.y = vi[1] * y[0] + vi[3] * y[1] + vi[4] * y[2];
      z.z = vi[2] * y[0] + vi[4] * y[1] + vi[5] * y[2];
      if (cur.pos0 >= 0) zq_cm[cur.pos0] = z;
      for (int jj = cur.b + l + G; jj < cur.e; jj += G) {
        const int pos = cp.pm_cm[jj];
        if (pos >= 0) zq_cm[pos] = z;
      }
    }
    cur = nxt;
  }
}

// Camera pass in the items of the BA camera pass: partial i = sum A_k zz_k over the item.
template <typename T>
__global__ void __launch_bounds__(kCamBlock)
k_gp_schur_cam(Compact<T> cp, const V4<T>* __restrict__ a_cm, const double* __restrict__ u,
               const P3<T>* __restrict__ zq_cm, CamItems it, int nslot,
               double* __restrict__ part, const PcgState* __restrict__ st) {
  if (st->done) return;
  const int4 rec = it.at[(blockIdx.x % it.R) * it.cap + blockIdx.x / it.R];
  if (rec.x < 0) return;
  const int Ca = cp.Ca;
  const int i = rec.x, s = rec.y, sb = rec.z, se = rec.w;
  __shared__ T smem[3 * (kCamBlock / kWave)];
  double us[3];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) us[c] = u[c * Ca + s];
  }
  T acc[3] = {T(0), T(0), T(0)};
#pragma unroll 2
  for (int k = sb + threadIdx.x; k < se; k += kCamBlock) {
    const P3<T> zv = zq_cm[k];
    const T z3[3] = {zv.x, zv.y, zv.z};
    T o[3];
    gp_apply(a_cm[k], z3, o);
    acc[0] += o[0];
    acc[1] += o[1];
    acc[2] += o[2];
  }
  block_sum<T, 3>(acc, smem);
  if (threadIdx.x == 0) {
    double pd = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = double(acc[c]);
      part[c * nslot + i] = v;
      pd += us[c] * v;
    }
    part[3 * nslot + i] = pd;
  }
}

template <typename T, int G>
__global__ void __launch_bounds__(kBlock)
k_gp_backsub(Compact<T> cp, const V4<T>* __restrict__ a_pm, const T* __restrict__ Vinv,
             const double* __restrict__ hp, const double* __restrict__ x,
             double* __restrict__ dp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = t / G;
  const int l = t % G;
  const int Ca = cp.Ca;
  double y[3] = {0.0, 0.0, 0.0};
  if (r < cp.Pa) {
    for (int j = cp.off[r] + l; j < cp.off[r + 1]; j += G) {
      const int s = cp.cam[j];
      if (s >= Ca) continue;
      const V4<T> a = a_pm[j];
      const double dc[3] = {x[s], x[Ca + s], x[2 * Ca + s]};
      const double ex = double(a.x) * dc[0] + double(a.y) * dc[1] + double(a.z) * dc[2];
      y[0] += double(a.w) * dc[0] - double(a.x) * ex;
      y[1] += double(a.w) * dc[1] - double(a.y) * ex;
      y[2] += double(a.w) * dc[2] - double(a.z) * ex;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) y[i] = group_sum<G>(y[i]);
  if (r >= cp.Pa || l != 0) return;
  double vi[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) vi[q] = double(Vinv[6 * r + q]);
  dp[3 * r] = hp[3 * r] + vi[0] * y[0] + vi[1] * y[1] + vi[2] * y[2];
  dp[3 * r + 1] = hp[3 * r + 1] + vi[1] * y[0] + vi[3] * y[1] + vi[4] * y[2];
  dp[3 * r + 2] = hp[3 * r + 2] + vi[2] * y[0] + vi[4] * y[1] + vi[5] * y[2];
}

// G lanes per point, each taking every G-th observation of the point's segment; the five
// sums are over observations, so the lanes need no combine step before the block sums.
template <typename T, int G>
__global__ void __launch_bounds__(kBlock)
k_gp_candidate(Compact<T> cp, const int* __restrict__ orig, const double* __restrict__ scales,
               double delta, double lam, double dmin, double dmax, const double* __restrict__ x,
               const double* __restrict__ dp, const double* __restrict__ gX,
               double* __restrict__ Xcand, double* __restrict__ s_cand,
               double* __restrict__ partials) {
  __shared__ double smem[5 * (kBlock / kWave)];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = t / G, l = t % G;
  const int Ca = cp.Ca;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // decrease, quad, g.delta, bad, cost'
  if (r < cp.Pa) {
    const double X[3] = {cp.Xd[3 * r], cp.Xd[3 * r + 1], cp.Xd[3 * r + 2]};
    const double dX[3] = {dp[3 * r], dp[3 * r + 1], dp[3 * r + 2]};
    const double Xn[3] = {X[0] + dX[0], X[1] + dX[1], X[2] + dX[2]};
    if (l == 0) {
      Xcand[3 * r] = Xn[0];
      Xcand[3 * r + 1] = Xn[1];
      Xcand[3 * r + 2] = Xn[2];
      acc[2] += gX[3 * r] * dX[0] + gX[3 * r + 1] * dX[1] + gX[3 * r + 2] * dX[2];
    }
    for (int j = cp.off[r] + l; j < cp.off[r + 1]; j += G) {
      const int s = cp.cam[j];
      const Cam<double> cm = cp.camd[s];
      const float dh = cp.depth[j];
      const GpObs o = gp_obs(cm, cp.xy[j], dh, X, dh > 0.0f ? 0.0 : scales[orig[j]]);
      double rho0, w, d2;
      huber(o.u[0] * o.u[0] + o.u[1] * o.u[1] + o.u[2] * o.u[2], delta, rho0, w, d2);
      double dc[3] = {0.0, 0.0, 0.0};
      if (s < Ca) {
        dc[0] = x[s];
        dc[1] = x[Ca + s];
        dc[2] = x[2 * Ca + s];
      }
      const double dd[3] = {dc[0] - dX[0], dc[1] - dX[1], dc[2] - dX[2]};
      double ds = 0.0;
      if (!o.pinned) {
        const double h = w * (o.d[0] * o.d[0] + o.d[1] * o.d[1] + o.d[2] * o.d[2]);
        const double hs = h + lam * fmin(fmax(h, dmin), dmax);
        const double gs = -w * (o.d[0] * o.u[0] + o.d[1] * o.u[1] + o.d[2] * o.u[2]);
        ds = (-gs + w * o.s * (o.d[0] * dd[0] + o.d[1] * dd[1] + o.d[2] * dd[2])) / hs;
        acc[2] += gs * ds;
      }
      const double sn = o.s + ds;
      s_cand[j] = sn;
      // model term at the linearisation point: J delta = s (dc - dX) - d ds
      double jd[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) jd[i] = o.s * dd[i] - o.d[i] * ds;
      acc[1] += w * (jd[0] * jd[0] + jd[1] * jd[1] + jd[2] * jd[2]);
      if (!o.pinned && !(sn > 0.0)) {
        acc[3] += 1.0;
      } else {
        double u2[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) u2[i] = o.v[i] - sn * (Xn[i] - (cm.c[i] + dc[i]));
        double rho, d1;
        huber(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2], delta, rho, d1, d2);
        acc[0] += 0.5 * (rho0 - rho);
        acc[4] += 0.5 * rho;
      }
    }
  }
  block_sum<double, 5>(acc, smem);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 5; ++i) partials[5 * blockIdx.x + i] = acc[i];
  }
}

__global__ void __launch_bounds__(kBlock)
k_gp_scatter(int Pa, int Ca, int64_t Nh, const int* __restrict__ pt_src,
             const double* __restrict__ Xcand, const int* __restrict__ cam_src,
             const double* __restrict__ x, const float* __restrict__ depth_hat,
             const int* __restrict__ orig, const double* __restrict__ s_cand,
             double* __restrict__ pts, double* __restrict__ cams, double* __restrict__ scales) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < Pa) {
    const int p = pt_src[i];
    pts[3 * p] = Xcand[3 * i];
    pts[3 * p + 1] = Xcand[3 * i + 1];
    pts[3 * p + 2] = Xcand[3 * i + 2];
  }
  if (i < Ca) {
    const int c = cam_src[i];
    cams[7 * c + 4] += x[i];
    cams[7 * c + 5] += x[Ca + i];
    cams[7 * c + 6] += x[2 * Ca + i];
  }
  if (i < Nh && !(depth_hat[i] > 0.0f)) scales[orig[i]] = s_cand[i];
}

inline unsigned blocks_for(int64_t n, int b = kBlock) { return unsigned((n + b - 1) / b); }

}  // namespace

// ================================================================== launchers
void launch_cam_table(hipStream_t s, int C, const double* cams, const double* intr,
                      Cam<double>* camd, Cam<float>* camf) {
  launch_k(k_cam_table, dim3(blocks_for(C)), dim3(kBlock), 0, s, C, cams, intr, camd,
                     camf);
}

void launch_validate(hipStream_t s, int64_t N, const Model& m, const int* pm_cam,
                     const int* pm_pt, const float2* xy, const float* depth,
                     const double* pts, const Cam<double>* camd, const int* inv_cm,
                     uint8_t* vrow, uint8_t* vrow_cm) {
  if (N == 0) return;
  launch_k(k_validate, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, m, pm_cam, pm_pt, xy, depth,
           pts, camd, inv_cm, vrow, vrow_cm);
}

void launch_validate_lds(hipStream_t s, int64_t N, int C, const Model& m, const int* pm_cam,
                         const int* pm_pt, const float2* xy, const float* depth,
                         const double* pts, const Cam<double>* camd, const int* inv_cm,
                         uint8_t* vrow, uint8_t* vrow_cm, const DevLimits& dl, int per_cu) {
  if (N == 0) return;
  const size_t tab = size_t(C) * sizeof(Cam<double>);
  bool use_lds = dl.n_cu > 0 && C > 0 && tab <= size_t(dl.lds_per_block);
  if (use_lds && tab > 65536)
    use_lds = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_validate_lds),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(tab)) ==
              hipSuccess;
  if (!use_lds) {
    launch_validate(s, N, m, pm_cam, pm_pt, xy, depth, pts, camd, inv_cm, vrow, vrow_cm);
    return;
  }
  const int64_t need = (N + kLdsWalkBlock - 1) / kLdsWalkBlock;
  const int grid = int(std::min<int64_t>(need, int64_t(dl.n_cu) * per_cu));
  launch_k(k_validate_lds, dim3(grid), dim3(kLdsWalkBlock), uint32_t(tab), s, N, C, m, pm_cam,
           pm_pt, xy, depth, pts, camd, inv_cm, vrow, vrow_cm);
}

void launch_cam_rows(hipStream_t s, int C, const int* cm_off, const uint8_t* vrow_cm,
                     const uint8_t* fixed, int need, uint8_t* act_c) {
  launch_k(k_cam_rows, dim3(C), dim3(kBlock), 0, s, cm_off, vrow_cm, fixed, need, act_c);
}

void launch_point_rows_prune(hipStream_t s, int P, const int* pt_off, const int* pm_cam,
                             const uint8_t* act_c, const uint8_t* fixed, int need,
                             const int* inv_cm, uint8_t* vrow, uint8_t* vrow_cm,
                             uint8_t* act_p, int* changed) {
  launch_k(k_point_rows_prune, dim3(blocks_for(P)), dim3(kBlock), 0, s, P, pt_off, pm_cam,
           act_c, fixed, need, inv_cm, vrow, vrow_cm, act_p, changed);
}

void launch_compact_points(hipStream_t s, int P, const uint8_t* act_p, const int* rank_p,
                           const int* pt_off, const int* pos_pm, const double* pts,
                           int* pt_src, int* off_hat, double* Xd, float* Xf) {
  launch_k(k_compact_points, dim3(blocks_for(P)), dim3(kBlock), 0, s, P, act_p,
                     rank_p, pt_off, pos_pm, pts, pt_src, off_hat, Xd, Xf);
}

void launch_compact_cams(hipStream_t s, int C, const uint8_t* act_c, const int* rank_c,
                         const uint8_t* fixed, const int* fixed_rank, const int* cm_off,
                         const int* pos_cm, int* slot_all, int* cam_src, int* cm_off_hat) {
  launch_k(k_compact_cams, dim3(blocks_for(C)), dim3(kBlock), 0, s, C, act_c, rank_c,
                     fixed, fixed_rank, cm_off, pos_cm, slot_all, cam_src, cm_off_hat);
}

void launch_compact_cam_table(hipStream_t s, int n, const int* cam_src,
                              const Cam<double>* camd, const Cam<float>* camf,
                              Cam<double>* camd_hat, Cam<float>* camf_hat) {
  if (n == 0) return;
  launch_k(k_compact_cam_table, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, cam_src,
                     camd, camf, camd_hat, camf_hat);
}

void launch_compact_obs(hipStream_t s, int64_t N, const uint8_t* vrow, const int* pos_pm,
                        const int* pm_cam, const int* slot_all, const float2* pm_xy,
                        const float* pm_depth, const int* pm_orig, int Ca, const int* inv_cm,
                        const int* pos_cm, const int* pm_pt, const int* rank_p, int* cam_hat,
                        float2* xy_hat, float* depth_hat, int* orig_hat, int* pm_cm,
                        int* cm_pt) {
  if (N == 0) return;
  launch_k(k_compact_obs, dim3((blocks_for(N) + 7) / 8 * 8), dim3(kBlock), 0, s, N, vrow,
           pos_pm, pm_cam,
           slot_all, pm_xy, pm_depth, pm_orig, Ca, inv_cm, pos_cm, pm_pt, rank_p, cam_hat,
           xy_hat, depth_hat, orig_hat, pm_cm, cm_pt);
}


// Lanes-per-point dispatch: G = 2, 4, 8 or 16 as a compile-time constant.
template <class F>
void with_lanes(int G, F&& f) {
  switch (G) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: f(std::integral_constant<int, 8>{});
  }
}

template <typename T, bool ADJ>
int lin_point_g(hipStream_t s, int G, const Model& m, const Compact<T>& cp, ObsMetric<T> om,
                double* V, double* gp, double* partials, const DevLimits& dl) {
  const size_t tab = size_t(cp.Ca + cp.Cf) * sizeof(Cam<double>);
  const bool lds = dl.n_cu > 0 && cp.Ca + cp.Cf > 0 && tab + 3 * 16 * 8 <= size_t(dl.lds_per_block);
  int nb = 0;
  with_lanes(G, [&](auto Gc) {
    constexpr int g = Gc();
    bool use = lds;
    if (use && tab > 65536)
      use = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lin_point<T, ADJ, g, 1024, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(tab)) == hipSuccess;
    if (use) {
      nb = lin_point_blocks_lds(cp.Pa);
      launch_k(k_lin_point<T, ADJ, g, 1024, true>, dim3(nb), dim3(1024), uint32_t(tab), s, m, cp,
               om, V, gp, partials);
    } else {
      nb = lin_point_blocks(cp.Pa);
      launch_k(k_lin_point<T, ADJ, g, kBlock, false>, dim3(nb), dim3(kBlock), 0, s, m, cp, om,
               V, gp, partials);
    }
  });
  return nb;
}

template <typename T>
int launch_lin_point(hipStream_t s, bool adj, int G, const Model& m, const Compact<T>& cp,
                     ObsMetric<T> om, double* V, double* gp, double* partials,
                     const DevLimits& dl) {
  if (adj) return lin_point_g<T, true>(s, G, m, cp, om, V, gp, partials, dl);
  return lin_point_g<T, false>(s, G, m, cp, om, V, gp, partials, dl);
}

template <typename T>
void launch_point_damp(hipStream_t s, int Pa, double lam, double dmin, double dmax,
                       const double* V, const double* gp, const double* rhs_p, T* Vinv,
                       double* hp, PtRec<T>* prec, int* bad) {
  launch_k(k_point_damp<T>, dim3(blocks_for(Pa)), dim3(kBlock), 0, s, Pa, lam, dmin, dmax, V,
           gp, rhs_p, Vinv, hp, prec, bad);
}

// Camera-dimension dispatch: D = 6 (pose) or 7 (pose and focal length); the adjoint mode
// exists for D = 6 only (the host rejects the other combination).
template <class F>
void with_dim(int D, F&& f) {
  if (D == 7)
    f(std::integral_constant<int, 7>{});
  else
    f(std::integral_constant<int, 6>{});
}

// Camera-pass grid: one workgroup per item slot up to the largest range's count (workgroups
// past their own range's last item return at once), so that the hardware hands items to CUs
// as they free up: item sizes vary by orders of magnitude (26.5 us against 31.4 us for a
// persistent grid of 8 workgroups per CU on the 1000-camera workload).
unsigned cam_grid(const CamItems& it, const DevLimits&) {
  return unsigned(std::max(1, std::min(it.slots, it.cap))) * unsigned(it.R);
}

template <typename T>
void launch_cam_items(hipStream_t s, bool adj, bool schur, int D, const Model& m,
                      const Compact<T>& cp, ObsMetric<T> om, const PtRec<T>* prec, CamItems it,
                      int nslot, double* part, const DevLimits& dl) {
  if (cp.Ca == 0 || nslot <= 0) return;
  const unsigned grid = cam_grid(it, dl);
  const dim3 block(cam_block<T>());
  if (adj) {
    if (schur)
      launch_k((k_cam_items<T, true, 6, true>), dim3(grid), block, 0, s, m, cp, om, prec, it,
               part);
    else
      launch_k((k_cam_items<T, true, 6, false>), dim3(grid), block, 0, s, m, cp, om, prec, it,
               part);
  } else {
    with_dim(D, [&](auto Dc) {
      if (schur)
        launch_k((k_cam_items<T, false, Dc(), true>), dim3(grid), block, 0, s, m, cp, om, prec,
                 it, part);
      else
        launch_k((k_cam_items<T, false, Dc(), false>), dim3(grid), block, 0, s, m, cp, om, prec,
                 it, part);
    });
  }
}

template <typename T>
void launch_cam_assemble(hipStream_t s, int D, int Ca, double lam, double dmin, double dmax,
                         const int* item_off, const double* part, const double* rhs_c,
                         double* Uraw, T* Ustar, double* gc, double* b, double* Minv,
                         double* Scc) {
  if (Ca == 0) return;
  with_dim(D, [&](auto Dc) {
    launch_k((k_cam_assemble<T, Dc()>), dim3(Ca), dim3(kBlock), 0, s, Ca, lam, dmin, dmax,
             item_off, part, rhs_c, Uraw, Ustar, gc, b, Minv, Scc);
  });
}

template <typename T>
void launch_mv_table(hipStream_t s, int D, int n, const Cam<double>* camd_hat, void* mvt) {
  if (n == 0) return;
  with_dim(D, [&](auto Dc) {
    launch_k(k_mv_table<T, Dc()>, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, camd_hat,
             static_cast<MvRec<T, Dc()>*>(mvt));
  });
}

// The PCG vector kernels also serve global positioning (D = 3).
template <class F>
void with_dim_pcg(int D, F&& f) {
  if (D == 3)
    f(std::integral_constant<int, 3>{});
  else
    with_dim(D, f);
}

void launch_range_bounds(hipStream_t s, int Ca, int R, int ppx, const int* cm_off,
                         const int* cm_pt, int* rb) {
  if (Ca <= 0 || R <= 1) return;
  launch_k(k_range_bounds, dim3(blocks_for(int64_t(Ca) * R)), dim3(kBlock), 0, s, Ca, R, ppx,
           cm_off, cm_pt, rb);
}

void launch_build_items(hipStream_t s, int Ca, const int* cm_off, const int* rb, int K,
                        CamItems it) {
  launch_k(k_build_items, dim3(1), dim3(1024), 0, s, Ca, cm_off, rb, K, it);
}

template <typename T>
void launch_pcg_init(hipStream_t s, int D, int Ca, const double* b, const double* Minv,
                     const T* Ustar, double* x, double* r, double* u, double* p, double* sv,
                     double* Uu, double* terms, void* mvt, PcgState* st, double tol2,
                     int max_iter) {
  with_dim_pcg(D, [&](auto Dc) {
    launch_k(k_pcg_init<T, Dc()>, dim3(1), dim3(1024), 0, s, Ca, b, Minv, Ustar, x, r, u, p, sv,
             Uu, terms, static_cast<MvRec<T, Dc()>*>(mvt), st, tol2, max_iter);
  });
}


template <typename T, bool ADJ, int G, int D>
void schur_point_launch(hipStream_t s, const Model& m, const Compact<T>& cp, ObsMetric<T> om,
                        const MvRec<T, D>* mvt, const T* Vinv, P3<T>* zq, const PcgState* st,
                        const DevLimits& dl) {
  const size_t tab = size_t(cp.Ca) * sizeof(MvRec<T, D>);
  bool use_lds = dl.n_cu > 0 && cp.Ca > 0 && tab <= size_t(dl.lds_per_block);
  const void* fn = reinterpret_cast<const void*>(&k_schur_point_lds<T, ADJ, G, D>);
  if (use_lds && tab > 65536)
    use_lds = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(tab)) ==
              hipSuccess;
  if (use_lds) {
    // float32 (80-byte records): two workgroups per CU share it (17.1 us against 19.3 us
    // with one on the 1000-camera workload). float64 (128-byte records, one workgroup per
    // CU): four workgroups per CU queued, so that CUs that finish early take more tiles.
    const int grid = (dl.n_cu * (sizeof(T) == 8 ? 4 : 2) + 7) / 8 * 8;
    const int ppx = (cp.Pa + 7) / 8;
    launch_k(k_schur_point_lds<T, ADJ, G, D>, dim3(grid), dim3(kPtLdsBlock), uint32_t(tab), s,
             m, cp, om, mvt, Vinv, zq, st, ppx);
  } else {
    const unsigned nb = (blocks_for(int64_t(cp.Pa) * G) + 7) / 8 * 8;   // one share per XCD
    launch_k(k_schur_point<T, ADJ, G, D>, dim3(nb), dim3(kBlock), 0, s, m, cp, om, mvt, Vinv,
             zq, st);
  }
}

template <typename T, bool ADJ, int D>
void schur_point_g(hipStream_t s, int G, const Model& m, const Compact<T>& cp, ObsMetric<T> om,
                   const MvRec<T, D>* mvt, const T* Vinv, P3<T>* zq, const PcgState* st,
                   const DevLimits& dl) {
  switch (G) {
    case 2: schur_point_launch<T, ADJ, 2, D>(s, m, cp, om, mvt, Vinv, zq, st, dl); break;
    case 4: schur_point_launch<T, ADJ, 4, D>(s, m, cp, om, mvt, Vinv, zq, st, dl); break;
    case 16: schur_point_launch<T, ADJ, 16, D>(s, m, cp, om, mvt, Vinv, zq, st, dl); break;
    default: schur_point_launch<T, ADJ, 8, D>(s, m, cp, om, mvt, Vinv, zq, st, dl);
  }
}

template <typename T>
void launch_schur_point(hipStream_t s, bool adj, int D, int G, const Model& m,
                        const Compact<T>& cp, ObsMetric<T> om, const void* mvt, const T* Vinv,
                        P3<T>* zq, const PcgState* st, const DevLimits& dl) {
  if (adj)
    schur_point_g<T, true, 6>(s, G, m, cp, om, static_cast<const MvRec<T, 6>*>(mvt), Vinv, zq,
                              st, dl);
  else
    with_dim(D, [&](auto Dc) {
      schur_point_g<T, false, Dc()>(s, G, m, cp, om, static_cast<const MvRec<T, Dc()>*>(mvt),
                                    Vinv, zq, st, dl);
    });
}

template <typename T>
void launch_schur_cam(hipStream_t s, bool adj, int D, const Model& m, const Compact<T>& cp,
                      ObsMetric<T> om, const double* u, const P3<T>* zq, CamItems it,
                      int nslot, double* part, const PcgState* st, const DevLimits& dl) {
  if (cp.Ca <= 0 || nslot <= 0) return;
  const unsigned grid = cam_grid(it, dl);
  const dim3 block(cam_block<T>());
  if (adj)
    launch_k((k_schur_cam<T, true, 6>), dim3(grid), block, 0, s, m, cp, om, u, zq, it, nslot,
             part, st);
  else
    with_dim(D, [&](auto Dc) {
      launch_k((k_schur_cam<T, false, Dc()>), dim3(grid), block, 0, s, m, cp, om, u, zq, it,
               nslot, part, st);
    });
}

template <typename T>
void launch_pcg_update(hipStream_t s, int D, int Ca, int k, const double* Minv, const T* Ustar,
                       const int* item_off, int nit, int nslot, const double* part,
                       double* terms, double* x, double* r, double* u, double* p, double* sv,
                       double* Uu, void* mvt, PcgState* st) {
  if (Ca <= 0) return;
  with_dim_pcg(D, [&](auto Dc) {
    launch_k(k_pcg_update<T, Dc()>, dim3((Ca + kUpdCams - 1) / kUpdCams), dim3(kUpdBlock), 0,
             s, Ca, k, Minv, Ustar, item_off, nit, nslot, part, terms, x, r, u, p, sv, Uu,
             static_cast<MvRec<T, Dc()>*>(mvt), st);
  });
}

template <typename T>
void launch_x_to_mv(hipStream_t s, int D, int Ca, const double* x, void* mvt, PcgState* st) {
  if (Ca <= 0) return;
  with_dim(D, [&](auto Dc) {
    launch_k(k_x_to_mv<T, Dc()>, dim3(blocks_for(Ca)), dim3(kBlock), 0, s, Ca, x,
             static_cast<MvRec<T, Dc()>*>(mvt), st);
  });
}

template <typename T>
void launch_true_residual(hipStream_t s, int D, int Ca, const double* x, const double* b,
                          const T* Ustar, const int* item_off, int nslot, const double* part,
                          double* out) {
  if (Ca <= 0) return;
  with_dim(D, [&](auto Dc) {
    launch_k(k_true_residual<T, Dc()>, dim3(1), dim3(1024), 0, s, Ca, x, b, Ustar, item_off,
             nslot, part, out);
  });
}

template <typename T>
void launch_backsub(hipStream_t s, int Pa, const double* hp, const P3<T>* zq, bool use_z,
                    double* dp) {
  if (Pa <= 0) return;
  launch_k(k_backsub<T>, dim3(blocks_for(Pa)), dim3(kBlock), 0, s, Pa, hp, zq, int(use_z), dp);
}

void launch_cam_candidate(hipStream_t s, int Ca, int Cf, int D, const int* cam_src,
                          const double* x, const double* cams, const Cam<double>* camd_hat,
                          double* cand_cams, Cam<double>* cand_tab) {
  if (Ca + Cf == 0) return;
  launch_k(k_cam_candidate, dim3(blocks_for(Ca + Cf)), dim3(kBlock), 0, s, Ca, Cf, D, cam_src,
           x, cams, camd_hat, cand_cams, cand_tab);
}

template <typename T, int G>
int point_candidate_g(hipStream_t s, const Model& m, const Compact<T>& cp, int D,
                      const Cam<double>* cand_tab, const double* x, const double* dp,
                      const double* gp, const T* w, double* Xcand, double* partials,
                      const DevLimits& dl) {
  const size_t tab = size_t(cp.Ca + cp.Cf) * sizeof(Cam<double>);
  bool lds = dl.n_cu > 0 && cp.Ca + cp.Cf > 0 && tab + 5 * 16 * 8 <= size_t(dl.lds_per_block);
  if (lds && tab > 65536)
    lds = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_point_candidate<T, G, 1024, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(tab)) == hipSuccess;
  if (lds) {
    const int nb = lin_point_blocks_lds(cp.Pa);
    launch_k(k_point_candidate<T, G, 1024, true>, dim3(nb), dim3(1024), uint32_t(tab), s, m, cp,
             D, cand_tab, x, dp, gp, w, Xcand, partials);
    return nb;
  }
  const int nb = lin_point_blocks(cp.Pa);
  launch_k(k_point_candidate<T, G, kBlock, false>, dim3(nb), dim3(kBlock), 0, s, m, cp, D,
           cand_tab, x, dp, gp, w, Xcand, partials);
  return nb;
}

// Two lanes per point: 107 us on the 1000-camera workload (eight observations per point)
// against 111, 117 and 131 us with 1, 4 and 8 lanes.
constexpr int kCandLanes = 2;

template <typename T>
int launch_point_candidate(hipStream_t s, const Model& m, const Compact<T>& cp, int D,
                           const Cam<double>* cand_tab, const double* x, const double* dp,
                           const double* gp, const T* w, double* Xcand, double* partials,
                           const DevLimits& dl) {
  if (cp.Pa <= 0) return 0;
  return point_candidate_g<T, kCandLanes>(s, m, cp, D, cand_tab, x, dp, gp, w, Xcand, partials,
                                          dl);
}

void launch_reduce_partials(hipStream_t s, int nblocks, int K, const double* partials,
                            unsigned max_mask, int ncu, const double* gc, const double* x,
                            double* out) {
  launch_k(k_reduce_partials, dim3(1), dim3(1024), 0, s, nblocks, K, partials, max_mask, ncu,
           gc, x, out);
}

void launch_scatter(hipStream_t s, int Pa, int Ca, const int* pt_src, const double* Xcand,
                    const int* cam_src, const double* cand_cams, const Cam<double>* cand_tab,
                    double* pts, double* cams, double* intr) {
  const int n = Pa > Ca ? Pa : Ca;
  if (n == 0) return;
  launch_k(k_scatter, dim3(blocks_for(n)), dim3(kBlock), 0, s, Pa, Ca, pt_src, Xcand, cam_src,
           cand_cams, cand_tab, pts, cams, intr);
}

void launch_adjoint_rhs(hipStream_t s, int Ca, int Pa, const int* cam_src, const double* cams,
                        const double* grad_cams, const int* pt_src, const int* pt_user,
                        const double* grad_pts, double* rhs_c, double* rhs_p) {
  const int n = Pa > Ca ? Pa : Ca;
  if (n == 0) return;
  launch_k(k_adjoint_rhs, dim3(blocks_for(n)), dim3(kBlock), 0, s, Ca, Pa, cam_src,
                     cams, grad_cams, pt_src, pt_user, grad_pts, rhs_c, rhs_p);
}

template <typename T>
void launch_adjoint_obs(hipStream_t s, const Model& m, const Compact<T>& cp, ObsMetric<T> om,
                        const double* x, const double* dp, const int* orig, float* gxy,
                        float* gdepth) {
  launch_k(k_adjoint_obs<T>, dim3(blocks_for(cp.Pa)), dim3(kBlock), 0, s, m, cp, om,
                     x, dp, orig, gxy, gdepth);
}

// explicit instantiations for the two precisions
#define IBA_INSTANTIATE(T)                                                                    \
  template int launch_lin_point<T>(hipStream_t, bool, int, const Model&, const Compact<T>&,   \
                                   ObsMetric<T>, double*, double*, double*, const DevLimits&); \
  template void launch_point_damp<T>(hipStream_t, int, double, double, double, const double*, \
                                     const double*, const double*, T*, double*, PtRec<T>*,    \
                                     int*);                                                    \
  template void launch_cam_items<T>(hipStream_t, bool, bool, int, const Model&,               \
                                    const Compact<T>&, ObsMetric<T>, const PtRec<T>*, CamItems,\
                                    int, double*, const DevLimits&);                           \
  template void launch_cam_assemble<T>(hipStream_t, int, int, double, double, double,         \
                                       const int*, const double*, const double*, double*, T*,  \
                                       double*, double*, double*, double*);                    \
  template void launch_mv_table<T>(hipStream_t, int, int, const Cam<double>*, void*);         \
  template void launch_pcg_init<T>(hipStream_t, int, int, const double*, const double*,       \
                                   const T*, double*, double*, double*, double*, double*,     \
                                   double*, double*, void*, PcgState*, double, int);           \
  template void launch_schur_point<T>(hipStream_t, bool, int, int, const Model&,              \
                                      const Compact<T>&, ObsMetric<T>, const void*, const T*, \
                                      P3<T>*, const PcgState*, const DevLimits&);              \
  template void launch_schur_cam<T>(hipStream_t, bool, int, const Model&, const Compact<T>&,  \
                                    ObsMetric<T>, const double*, const P3<T>*, CamItems, int, \
                                    double*, const PcgState*, const DevLimits&);              \
  template void launch_pcg_update<T>(hipStream_t, int, int, int, const double*, const T*,     \
                                     const int*, int, int, const double*, double*, double*,   \
                                     double*, double*, double*, double*, double*, void*,      \
                                     PcgState*);                                               \
  template void launch_x_to_mv<T>(hipStream_t, int, int, const double*, void*, PcgState*);    \
  template void launch_true_residual<T>(hipStream_t, int, int, const double*, const double*,  \
                                        const T*, const int*, int, const double*, double*);   \
  template void launch_backsub<T>(hipStream_t, int, const double*, const P3<T>*, bool,        \
                                  double*);                                                    \
  template int launch_point_candidate<T>(hipStream_t, const Model&, const Compact<T>&, int,   \
                                         const Cam<double>*, const double*, const double*,    \
                                         const double*, const T*, double*, double*,           \
                                         const DevLimits&);                                   \
  template void launch_adjoint_obs<T>(hipStream_t, const Model&, const Compact<T>&,           \
                                      ObsMetric<T>, const double*, const double*, const int*, \
                                      float*, float*);

IBA_INSTANTIATE(float)
IBA_INSTANTIATE(double)

// ------------------------------------------------------------------ explicit system launchers
template <typename T>
void launch_pair_counts(hipStream_t s, const Compact<T>& cp, int64_t* cnt, int* pm_rank) {
  if (cp.Pa == 0) return;
  launch_k(k_pair_counts<T>, dim3(blocks_for(cp.Pa)), dim3(kBlock), 0, s, cp, cnt, pm_rank);
}

template <typename T>
void launch_pair_keys(hipStream_t s, const Compact<T>& cp, const int64_t* coff, uint32_t* key,
                      uint64_t* val) {
  if (cp.Pa == 0) return;
  constexpr int G = 8;
  launch_k(k_pair_keys<T, G>, dim3(blocks_for(int64_t(cp.Pa) * G)), dim3(kBlock), 0, s, cp,
           coff, key, val);
}

void launch_run_flags(hipStream_t s, int64_t n, const uint32_t* key, int64_t* flag) {
  if (n == 0) return;
  launch_k(k_run_flags, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, key, flag);
}

void launch_block_list(hipStream_t s, int64_t n, const uint32_t* key, const int64_t* flag,
                       const int64_t* bidx, uint32_t* bkey, int64_t* bstart) {
  if (n == 0) return;
  launch_k(k_block_list, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, key, flag, bidx, bkey,
           bstart);
}

void launch_block_rows(hipStream_t s, int Ca, int64_t nb, const uint32_t* bkey, int64_t* row_ptr) {
  launch_k(k_block_rows, dim3(blocks_for(int64_t(Ca) + 1)), dim3(kBlock), 0, s, Ca, nb, bkey,
           row_ptr);
}

template <typename T>
void launch_schur_blocks(hipStream_t s, int D, const Model& m, const Compact<T>& cp,
                         ObsMetric<T> om, const T* Vinv, const int* pm_rank, int64_t nb,
                         const uint32_t* bkey, const int64_t* bstart, const uint64_t* sval,
                         T* sblk) {
  if (nb == 0) return;
  with_dim(D, [&](auto Dc) {
    launch_k(k_schur_blocks<T, Dc()>, dim3(blocks_for(nb * kWave)), dim3(kBlock), 0, s, m, cp,
             om, Vinv, pm_rank, nb, bkey, bstart, sval, sblk);
  });
}

template <typename T>
void launch_schur_spmv(hipStream_t s, int D, int Ca, const int64_t* row_ptr,
                       const uint32_t* bkey, const T* sblk, const double* Scc, const double* u,
                       const double* Uu, int nslot, double* part, const PcgState* st) {
  if (Ca == 0) return;
  with_dim(D, [&](auto Dc) {
    launch_k(k_schur_spmv<T, Dc()>, dim3(blocks_for(int64_t(Ca) * kWave)), dim3(kBlock), 0, s,
             Ca, row_ptr, bkey, sblk, Scc, u, Uu, nslot, part, st);
  });
}

#define IBA_EXPLICIT_INSTANTIATE(T)                                                            \
  template void launch_pair_counts<T>(hipStream_t, const Compact<T>&, int64_t*, int*);        \
  template void launch_pair_keys<T>(hipStream_t, const Compact<T>&, const int64_t*, uint32_t*, \
                                    uint64_t*);                                               \
  template void launch_schur_blocks<T>(hipStream_t, int, const Model&, const Compact<T>&,     \
                                       ObsMetric<T>, const T*, const int*, int64_t,           \
                                       const uint32_t*, const int64_t*, const uint64_t*, T*); \
  template void launch_schur_spmv<T>(hipStream_t, int, int, const int64_t*, const uint32_t*,  \
                                     const T*, const double*, const double*, const double*,   \
                                     int, double*, const PcgState*);

IBA_EXPLICIT_INSTANTIATE(float)
IBA_EXPLICIT_INSTANTIATE(double)

// ------------------------------------------------------------------ global positioning launchers
void launch_gp_validate(hipStream_t s, int64_t N, const float2* pm_xy, const float* pm_depth,
                        const int* inv_cm, uint8_t* vrow, uint8_t* vrow_cm) {
  if (N == 0) return;
  launch_k(k_gp_validate, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, pm_xy, pm_depth, inv_cm,
           vrow, vrow_cm);
}

void launch_gp_init_scales(hipStream_t s, int64_t N, const int* pm_cam, const int* pm_pt,
                           const int* pm_orig, const float2* pm_xy, const float* pm_depth,
                           const double* pts, const Cam<double>* camd, double* scales) {
  if (N == 0) return;
  launch_k(k_gp_init_scales, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, pm_cam, pm_pt, pm_orig,
           pm_xy, pm_depth, pts, camd, scales);
}

template <typename T>
int launch_gp_lin(hipStream_t s, int G, const Compact<T>& cp, const int* orig,
                  const double* scales, double delta, GpLin<T>* lin_pm, GpLin<T>* lin_cm,
                  double* gX, double* partials, const DevLimits& dl) {
  const size_t tab = size_t(cp.Ca + cp.Cf) * sizeof(Cam<double>);
  const bool lds = dl.n_cu > 0 && cp.Ca + cp.Cf > 0 && tab + 3 * 16 * 8 <= size_t(dl.lds_per_block);
  int nb = 0;
  with_lanes(G, [&](auto Gc) {
    constexpr int g = Gc();
    bool use = lds;
    if (use && tab > 65536)
      use = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gp_lin<T, g, 1024, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(tab)) == hipSuccess;
    if (use) {
      nb = lin_point_blocks_lds(cp.Pa);
      launch_k(k_gp_lin<T, g, 1024, true>, dim3(nb), dim3(1024), uint32_t(tab), s, cp, orig,
               scales, delta, lin_pm, lin_cm, gX, partials);
    } else {
      nb = lin_point_blocks(cp.Pa);
      launch_k(k_gp_lin<T, g, kBlock, false>, dim3(nb), dim3(kBlock), 0, s, cp, orig, scales,
               delta, lin_pm, lin_cm, gX, partials);
    }
  });
  return nb;
}

template <typename T>
void launch_gp_point_setup(hipStream_t s, int G, const Compact<T>& cp, double lam, double dmin,
                           double dmax, const GpLin<T>* lin_pm, V4<T>* a_pm, V4<T>* a_cm,
                           T* Vinv, double* hp, PtRec<T>* prec, int* bad) {
  if (cp.Pa == 0) return;
  with_lanes(G, [&](auto Gc) {
    launch_k(k_gp_point_setup<T, Gc()>, dim3(blocks_for(int64_t(cp.Pa) * Gc())), dim3(kBlock),
             0, s, cp, lam, dmin, dmax, lin_pm, a_pm, a_cm, Vinv, hp, prec, bad);
  });
}

template <typename T>
void launch_gp_cam_assemble(hipStream_t s, const Compact<T>& cp, double lam, double dmin,
                            double dmax, const GpLin<T>* lin_cm, const V4<T>* a_cm,
                            const PtRec<T>* prec, T* Ustar, double* gc, double* b,
                            double* Minv) {
  if (cp.Ca == 0) return;
  launch_k(k_gp_cam_assemble<T>, dim3(cp.Ca), dim3(kBlock), 0, s, cp, lam, dmin, dmax, lin_cm,
           a_cm, prec, Ustar, gc, b, Minv);
}

template <typename T>
void launch_gp_schur_point(hipStream_t s, int G, const Compact<T>& cp, const V4<T>* a_pm,
                           const void* mvt, const T* Vinv, P3<T>* zq_cm, const PcgState* st,
                           const DevLimits& dl) {
  if (cp.Pa == 0) return;
  const size_t tab = size_t(cp.Ca) * sizeof(GpMv<T>);
  with_lanes(G, [&](auto Gc) {
    // float32: the LDS kernel with one workgroup per CU (33.8 us against 35.8 us per point on
    // the 1000-camera workload; 44.5 us with two per CU); float64: one thread group per
    // point (97.8 us against 114 us)
    bool use_lds = sizeof(T) == 4 && dl.n_cu > 0 && cp.Ca > 0 &&
                   tab <= size_t(dl.lds_per_block);
    if (use_lds && tab > 65536)
      use_lds = hipFuncSetAttribute(
                    reinterpret_cast<const void*>(&k_gp_schur_point_lds<T, Gc()>),
                    hipFuncAttributeMaxDynamicSharedMemorySize, int(tab)) == hipSuccess;
    if (use_lds) {
      const int grid = (dl.n_cu + 7) / 8 * 8;
      const int ppx = (cp.Pa + 7) / 8;
      launch_k(k_gp_schur_point_lds<T, Gc()>, dim3(grid), dim3(kPtLdsBlock), uint32_t(tab), s,
               cp, a_pm, static_cast<const GpMv<T>*>(mvt), Vinv, zq_cm, st, ppx);
    } else {
      const unsigned nb = (blocks_for(int64_t(cp.Pa) * Gc()) + 7) / 8 * 8;
      launch_k(k_gp_schur_point<T, Gc()>, dim3(nb), dim3(kBlock), 0, s, cp, a_pm,
               static_cast<const GpMv<T>*>(mvt), Vinv, zq_cm, st);
    }
  });
}

template <typename T>
void launch_gp_schur_cam(hipStream_t s, const Compact<T>& cp, const V4<T>* a_cm,
                         const double* u, const P3<T>* zq_cm, CamItems it, int nslot,
                         double* part, const PcgState* st, const DevLimits& dl) {
  if (cp.Ca <= 0 || nslot <= 0) return;
  launch_k(k_gp_schur_cam<T>, dim3(cam_grid(it, dl)), dim3(kCamBlock), 0, s, cp, a_cm, u,
           zq_cm, it, nslot, part, st);
}

template <typename T>
void launch_gp_backsub(hipStream_t s, int G, const Compact<T>& cp, const V4<T>* a_pm,
                       const T* Vinv, const double* hp, const double* x, double* dp) {
  if (cp.Pa == 0) return;
  with_lanes(G, [&](auto Gc) {
    launch_k(k_gp_backsub<T, Gc()>, dim3(blocks_for(int64_t(cp.Pa) * Gc())), dim3(kBlock), 0, s,
             cp, a_pm, Vinv, hp, x, dp);
  });
}

template <typename T>
int launch_gp_candidate(hipStream_t s, int G, const Compact<T>& cp, const int* orig,
                        const double* scales, double delta, double lam, double dmin,
                        double dmax, const double* x, const double* dp, const double* gX,
                        double* Xcand, double* s_cand, double* partials, const DevLimits& dl) {
  if (cp.Pa == 0) return 0;
  // the camera table stays in L2 here: staging it in LDS gave no gain (170 against 173 us)
  (void)dl;
  int nb = 0;
  with_lanes(G, [&](auto Gc) {
    nb = int(blocks_for(int64_t(cp.Pa) * Gc()));
    launch_k(k_gp_candidate<T, Gc()>, dim3(nb), dim3(kBlock), 0, s, cp, orig, scales, delta,
             lam, dmin, dmax, x, dp, gX, Xcand, s_cand, partials);
  });
  return nb;
}

void launch_gp_scatter(hipStream_t s, int Pa, int Ca, int64_t Nh, const int* pt_src,
                       const double* Xcand, const int* cam_src, const double* x,
                       const float* depth_hat, const int* orig, const double* s_cand,
                       double* pts, double* cams, double* scales) {
  const int64_t n = std::max<int64_t>(Nh, std::max(Pa, Ca));
  if (n == 0) return;
  launch_k(k_gp_scatter, dim3(blocks_for(n)), dim3(kBlock), 0, s, Pa, Ca, Nh, pt_src, Xcand,
           cam_src, x, depth_hat, orig, s_cand, pts, cams, scales);
}

#define IBA_GP_INSTANTIATE(T)                                                                  \
  template int launch_gp_lin<T>(hipStream_t, int, const Compact<T>&, const int*,              \
                                const double*, double, GpLin<T>*, GpLin<T>*, double*,         \
                                double*, const DevLimits&);                                   \
  template void launch_gp_point_setup<T>(hipStream_t, int, const Compact<T>&, double, double, \
                                         double, const GpLin<T>*, V4<T>*, V4<T>*, T*, double*,\
                                         PtRec<T>*, int*);                                     \
  template void launch_gp_cam_assemble<T>(hipStream_t, const Compact<T>&, double, double,     \
                                          double, const GpLin<T>*, const V4<T>*,              \
                                          const PtRec<T>*, T*, double*, double*, double*);    \
  template void launch_gp_schur_point<T>(hipStream_t, int, const Compact<T>&, const V4<T>*,   \
                                         const void*, const T*, P3<T>*, const PcgState*,      \
                                         const DevLimits&);                                   \
  template void launch_gp_schur_cam<T>(hipStream_t, const Compact<T>&, const V4<T>*,          \
                                       const double*, const P3<T>*, CamItems, int, double*,   \
                                       const PcgState*, const DevLimits&);                    \
  template void launch_gp_backsub<T>(hipStream_t, int, const Compact<T>&, const V4<T>*,       \
                                     const T*, const double*, const double*, double*);        \
  template int launch_gp_candidate<T>(hipStream_t, int, const Compact<T>&, const int*,        \
                                      const double*, double, double, double, double,          \
                                      const double*, const double*, const double*, double*,   \
                                      double*, double*, const DevLimits&);

IBA_GP_INSTANTIATE(float)
IBA_GP_INSTANTIATE(double)


void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
}

int64_t launches_issued() { return g_launches; }

}  // namespace iba
