// Shared device-side definitions of the mcproj HIP library (gfx950).
//
// Layout of a problem on the device (DevProblem): one struct in global memory
// holding every per-scene constant in FP64 (residual precision) and FP32 (step
// precision). All kernel accesses to it use wave-uniform addresses, so they
// compile to scalar loads that stay in the scalar cache.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace mc {

constexpr int MAXJ = 36;    // joints (= DoF of kinematic families)
constexpr int MAXF = 4;     // end-effector frames
constexpr int MAXB = 4;     // constraint blocks
constexpr int MAXM = 20;    // stacked rows
constexpr int MAXS = 320;   // robot collision spheres
constexpr int LIN_D = 8;    // linear family: padded d
constexpr int LIN_M = 6;    // linear family: padded m

enum : int { REV = 0, PRI = 1 };
enum : int { B_POSE = 0, B_REL = 1, B_AXIS = 2, B_COM = 3, B_SPHERE = 4, B_LINEAR = 5 };
enum : int { ST_CONVERGED = 0, ST_MAX_ITER = 1, ST_SINGULAR = 2, ST_DIVERGED = 3, ST_NONFINITE = 4 };
enum : int { V_FREE = 0, V_HIT = 1, V_UNCHECKED = 2 };

template <class T>
struct TP {
  T jR[MAXJ][9];       // joint origin rotation (row-major)
  T jp[MAXJ][3];       // joint origin translation
  T fR[MAXF][9];       // end-effector frame offset rotation
  T fp[MAXF][3];       // end-effector frame offset translation
  T refRt[MAXB][9];    // R_ref^T of pose / relative-pose blocks
  T refp[MAXB][3];     // p_ref
  T target[MAXB][3];   // centre-of-mass target (x, y)
  T mass[MAXJ];        // link masses
  T mcom[MAXJ][3];     // mass * local centre of mass
  T submass[MAXJ];     // mass of the subtree rooted at joint j
  T inv_total_mass;
  T A[LIN_M][LIN_D];   // linear family (zero padded)
  T b[LIN_M];
};

struct DevProblem {
  TP<double> d;
  TP<float> f;
  int32_t dof, rows, family, lin_d, lin_m;
  int32_t n_sph, n_obs, n_clus;
  int32_t sph_begin[MAXJ + 1];   // spheres of link l: [sph_begin[l], sph_begin[l+1])
  float4 sph[MAXS];              // local centre, radius
  float4 link_bs[MAXJ];          // link bounding sphere: local centre, radius (inflated), w<0: none
  float4 point_sph;              // sphere family: offset and radius of the point robot
  const float4* obs;             // obstacles (x, y, z, r), grouped by cluster
  const float4* clus;            // cluster bounding spheres (centre, inflated radius)
  const int2* clus_range;        // obstacle index range of each cluster
  unsigned long long* fallback_counter;
};

template <class T> __device__ __forceinline__ const TP<T>& tp(const DevProblem& P);
template <> __device__ __forceinline__ const TP<double>& tp<double>(const DevProblem& P) { return P.d; }
template <> __device__ __forceinline__ const TP<float>& tp<float>(const DevProblem& P) { return P.f; }

// ---------------------------------------------------------------- compile-time loops
template <int N> using ic = std::integral_constant<int, N>;

template <int I, int N, class F>
__host__ __device__ __forceinline__ void sfor(F&& f) {
  if constexpr (I < N) {
    f(ic<I>{});
    sfor<I + 1, N>(f);
  }
}

// ---------------------------------------------------------------- small math
template <class T> struct Rig { T R[9]; T p[3]; };

// FP64 sine and cosine for moderate arguments (|x| < 1e5, joint angles), a few ulp accurate:
// Cody-Waite reduction x = k pi/2 + r with pi/2 split into three doubles (hi + mid + lo),
// then the Taylor series of sin (to r^15) and cos (to r^16) on |r| <= pi/4, whose
// truncation errors are below 5e-17. No large-argument path.
__device__ __forceinline__ void sincos_t(double x, double* s, double* c) {
  const double k = __builtin_rint(x * 0.6366197723675814);
  double r = __builtin_fma(-k, 1.5707963267948966, x);
  r = __builtin_fma(-k, 6.123233995736766e-17, r);
  r = __builtin_fma(-k, -1.4973849048591698e-33, r);
  const double r2 = r * r;
  double ps = -1.0 / 1307674368000.0;
  ps = __builtin_fma(ps, r2, 1.0 / 6227020800.0);
  ps = __builtin_fma(ps, r2, -1.0 / 39916800.0);
  ps = __builtin_fma(ps, r2, 1.0 / 362880.0);
  ps = __builtin_fma(ps, r2, -1.0 / 5040.0);
  ps = __builtin_fma(ps, r2, 1.0 / 120.0);
  ps = __builtin_fma(ps, r2, -1.0 / 6.0);
  const double sn = __builtin_fma(ps * r2, r, r);
  double pc = 1.0 / 20922789888000.0;
  pc = __builtin_fma(pc, r2, -1.0 / 87178291200.0);
  pc = __builtin_fma(pc, r2, 1.0 / 479001600.0);
  pc = __builtin_fma(pc, r2, -1.0 / 3628800.0);
  pc = __builtin_fma(pc, r2, 1.0 / 40320.0);
  pc = __builtin_fma(pc, r2, -1.0 / 720.0);
  pc = __builtin_fma(pc, r2, 1.0 / 24.0);
  pc = __builtin_fma(pc, r2, -0.5);
  const double cs = __builtin_fma(pc, r2, 1.0);
  const int qd = int(k) & 3;  // quadrant
  const double s0 = (qd & 1) ? cs : sn;
  const double c0 = (qd & 1) ? sn : cs;
  *s = (qd & 2) ? -s0 : s0;
  *c = ((qd + 1) & 2) ? -c0 : c0;
}
__device__ __forceinline__ void sincos_t(float x, float* s, float* c) { __sincosf(x, s, c); }
__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt(x); }
__device__ __forceinline__ float rsqrt_t(float x) { return __frsqrt_rn(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_t(float x) { return __fsqrt_rn(x); }
__device__ __forceinline__ bool finite_t(double x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool finite_t(float x) { return __builtin_isfinite(x); }

// Opaque copy: stops the compiler from proving two recomputations equal (and
// merging them, which would keep every intermediate live across the solve).
__device__ __forceinline__ float opaque(float x) { asm volatile("" : "+v"(x)); return x; }
__device__ __forceinline__ double opaque(double x) { asm volatile("" : "+v"(x)); return x; }

// Problem constants for one pass: the pointer is moved to the constant address space, so
// the loads become scalar (s_load) reads, and passed through an opaque barrier, so they are
// re-issued per pass instead of being hoisted out of the Newton loop into registers.
// The pointer is wave-uniform by construction; readfirstlane states it (out-of-line
// functions cannot prove it) so it can live in scalar registers.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
  return reinterpret_cast<T*>((uint64_t(hi) << 32) | lo);
}
using cDevProblem = const __attribute__((address_space(4))) DevProblem;
__device__ __forceinline__ const DevProblem& cparams(const DevProblem* p) {
  cDevProblem* c = (cDevProblem*)uniform_ptr(p);
  asm volatile("" : "+s"(c));
  return *(const DevProblem*)c;
}

// Ordering helpers for the unrolled kinematic chains: an empty asm that claims to read `dep`
// and rewrite `x`, so x (and everything computed from it, e.g. a joint's sine and cosine or
// the loads of its origin) cannot be scheduled before dep exists. Costs no instruction; keeps
// the register footprint of a tree walk to the frames actually in flight.
template <class T, class U>
__device__ __forceinline__ T after(T x, U dep) {
  asm volatile("" : "+v"(x) : "v"(dep));
  return x;
}
template <class TPT, class U>
__device__ __forceinline__ const TPT& after_params(const TPT& P, U dep) {
  using cT = const __attribute__((address_space(4))) TPT;
  cT* c = (cT*)uniform_ptr(&P);
  asm volatile("" : "+s"(c) : "v"(dep));
  return *(const TPT*)c;
}
template <class T, class U, class V>
__device__ __forceinline__ T after2(T x, U d0, V d1) {
  asm volatile("" : "+v"(x) : "v"(d0), "v"(d1));
  return x;
}

// Accessors for the FP64 iterate. at(j) returns coordinate j; at(j, dep) issues the read only
// after dep exists. Reads go through an opaque copy so separate passes never share them.
struct QLds {  // per-lane column in LDS: q[j] at base[j * stride]
  double* base;
  int stride;
  __device__ __forceinline__ double at(int j) const { return opaque(base[j * stride]); }
  template <class U>
  __device__ __forceinline__ double at(int j, U dep) const { return opaque(base[after(j * stride, dep)]); }
  __device__ __forceinline__ void set(int j, double v) const { base[j * stride] = v; }
};
template <class T>
struct QArr {  // registers
  const T* q;
  __device__ __forceinline__ double at(int j) const { return double(opaque(q[j])); }
  template <class U>
  __device__ __forceinline__ double at(int j, U dep) const { return double(after(q[j], dep)); }
};

constexpr int pidx(int i, int k) { return i * (i + 1) / 2 + k; }  // packed lower triangle, i >= k

template <class T>
__device__ __forceinline__ void cross3(const T* a, const T* b, T* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
template <class T>
__device__ __forceinline__ void matvec3(const T* M, const T* v, T* o) {
  o[0] = M[0] * v[0] + M[1] * v[1] + M[2] * v[2];
  o[1] = M[3] * v[0] + M[4] * v[1] + M[5] * v[2];
  o[2] = M[6] * v[0] + M[7] * v[1] + M[8] * v[2];
}
// o = M^T v
template <class T>
__device__ __forceinline__ void matTvec3(const T* M, const T* v, T* o) {
  o[0] = M[0] * v[0] + M[3] * v[1] + M[6] * v[2];
  o[1] = M[1] * v[0] + M[4] * v[1] + M[7] * v[2];
  o[2] = M[2] * v[0] + M[5] * v[1] + M[8] * v[2];
}
// C = A B
template <class T>
__device__ __forceinline__ void matmul3(const T* A, const T* B, T* C) {
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) C[3 * i + k] = A[3 * i] * B[k] + A[3 * i + 1] * B[3 + k] + A[3 * i + 2] * B[6 + k];
}
// C = A^T B
template <class T>
__device__ __forceinline__ void matTmul3(const T* A, const T* B, T* C) {
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) C[3 * i + k] = A[i] * B[k] + A[3 + i] * B[3 + k] + A[6 + i] * B[6 + k];
}

// SO(3) log (vee form) of R plus the left-Jacobian inverse J_l^-1(w), used for the angular
// rows of the pose errors: v = vee(R - R^T)/2 = sin(theta) * axis, c = cos(theta),
// w = (theta / sin theta) v, with the first-order Taylor form 1 + s^2/6 of theta/sin(theta)
// near theta = 0 (Sec. IV-A). For a left perturbation R' = exp([e]x) R,
// d log(R') / d e = J_l^-1(w) = I - [w]x / 2 + beta [w]x^2, beta = 1/theta^2 - (1 + c)/(2 theta s).
__device__ __forceinline__ void so3_log_jlinv(const double* R, double* w, double* Jinv) {
  const double v0 = 0.5 * (R[7] - R[5]), v1 = 0.5 * (R[2] - R[6]), v2 = 0.5 * (R[3] - R[1]);
  const double s2 = v0 * v0 + v1 * v1 + v2 * v2;
  const double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
  double f;
  if (c > 0.0 && s2 < 1e-8) {
    f = 1.0 + s2 * (1.0 / 6.0);
  } else if (c > 0.0 && s2 < 1e-2) {
    // theta < pi/2: theta / sin(theta) = asin(s) / s = sum_n C(2n, n) s^2n / (4^n (2n + 1))
    f = 6435.0 / 557056.0;
    f = __builtin_fma(f, s2, 143.0 / 10240.0);
    f = __builtin_fma(f, s2, 231.0 / 13312.0);
    f = __builtin_fma(f, s2, 63.0 / 2816.0);
    f = __builtin_fma(f, s2, 35.0 / 1152.0);
    f = __builtin_fma(f, s2, 5.0 / 112.0);
    f = __builtin_fma(f, s2, 3.0 / 40.0);
    f = __builtin_fma(f, s2, 1.0 / 6.0);
    f = __builtin_fma(f, s2, 1.0);
  } else {
    const double sn = sqrt(s2);
    f = atan2(sn, c) / sn;
  }
  w[0] = f * v0; w[1] = f * v1; w[2] = f * v2;
  if (Jinv) {
    const double th2 = f * f * s2;
    double beta;
    if (th2 < 0.1) {
      // 1/theta^2 - cot(theta/2) / (2 theta) = 1/12 + th^2/720 + th^4/30240 + th^6/1209600 + th^8/47900160 + ...
      beta = 1.0 / 47900160.0;
      beta = __builtin_fma(beta, th2, 1.0 / 1209600.0);
      beta = __builtin_fma(beta, th2, 1.0 / 30240.0);
      beta = __builtin_fma(beta, th2, 1.0 / 720.0);
      beta = __builtin_fma(beta, th2, 1.0 / 12.0);
    } else {
      const double th = sqrt(th2), sn = sqrt(s2);
      beta = 1.0 / th2 - (1.0 + c) / (2.0 * th * sn);
    }
    const double a0 = 1.0 - beta * th2;
    // J = a0 I - 0.5 [w]x + beta w w^T
    Jinv[0] = a0 + beta * w[0] * w[0];
    Jinv[1] = 0.5 * w[2] + beta * w[0] * w[1];
    Jinv[2] = -0.5 * w[1] + beta * w[0] * w[2];
    Jinv[3] = -0.5 * w[2] + beta * w[1] * w[0];
    Jinv[4] = a0 + beta * w[1] * w[1];
    Jinv[5] = 0.5 * w[0] + beta * w[1] * w[2];
    Jinv[6] = 0.5 * w[1] + beta * w[2] * w[0];
    Jinv[7] = -0.5 * w[0] + beta * w[2] * w[1];
    Jinv[8] = a0 + beta * w[2] * w[2];
  }
}

}  // namespace mc
