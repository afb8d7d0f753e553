// Shared device-side definitions of the mcproj HIP library (gfx950).
//
// Data layout. A problem lives in global memory as one DevProblem. Its kinematic and
// constraint constants (Consts: FP64 copy for the residual pass, FP32 copy for the step
// passes) and its collision constants (CollConsts; obstacles follow in a separate array) are
// wave-uniform: the projection kernels read them with scalar loads (through the constant
// address space, into scalar registers), each joint's data requested one joint ahead of its
// use along the kinematic walk; the exact-check kernels stage the robot spheres and obstacles
// in LDS per workgroup. A lane's FP64 iterate is a column of a per-wave [D][64] LDS tile.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace mc {

constexpr int MAXJ = 36;    // joints (= DoF of kinematic families)
constexpr int MAXF = 8;     // end-effector frames
constexpr int MAXB = 6;     // constraint blocks
constexpr int MAXM = 22;    // stacked rows
constexpr int MAXHV = 8;    // support-polygon vertices
constexpr int MAXS = 320;   // robot collision spheres
constexpr int MAXC = 128;   // obstacle clusters
constexpr int MAXO = 2048;  // obstacle spheres
constexpr int LIN_D = 8;    // linear family: padded d
constexpr int LIN_M = 6;    // linear family: padded m

enum : int { REV = 0, PRI = 1 };
enum : int { B_POSE = 0, B_REL = 1, B_AXIS = 2, B_COM = 3, B_SPHERE = 4, B_LINEAR = 5, B_DIST = 6, B_HULL = 7 };
constexpr int BF_BOUNDED = 1;  // POSE block flag: rows are the excess over finite bounds
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
  T target[MAXB][3];   // centre-of-mass target (x, y); rod length (closed-linkage blocks)
  T blo[MAXB][6];      // bounded pose blocks: lower and upper bound of each component of [t; log(R)^v]
  T bhi[MAXB][6];
  T hull_e[MAXHV][4];  // support polygon edge i: start vertex (x, y) and edge vector (x, y)
  T hull_n[MAXHV][4];  // its outward unit normal (x, y) and 1 / |edge|^2
  T mass[MAXJ];        // link masses
  T mcom[MAXJ][3];     // mass * local centre of mass
  T submass[MAXJ];     // mass of the subtree rooted at joint j
  T inv_total_mass;
  T A[LIN_M][LIN_D];   // linear family (zero padded)
  T b[LIN_M];
  float lbs[MAXJ][4];  // link bounding sphere (local centre, inflated radius; radius < 0: none)
  float obs_lo[4];     // box bounding all obstacle spheres (inflated; empty box without obstacles)
  float obs_hi[4];
};

// Kinematic and constraint constants (read by the kernels with scalar loads).
struct alignas(16) Consts {
  TP<double> d;
  TP<float> f;
  int32_t dof, rows, lin_m, hull_nv;
};

constexpr int MAXSUP = 32;  // groups of obstacle clusters

// Collision data. Obstacles are grouped by a recursive median split into clusters of at most 16
// spheres, and consecutive clusters into groups of at most 8; both levels carry an axis-aligned
// box that bounds their spheres (inflated by a small margin), and each robot link a bounding
// sphere of its own spheres.
struct alignas(16) CollConsts {
  int32_t n_sph, n_obs, n_clus, n_sup;
  int32_t sph_begin[MAXJ + 4];   // spheres of link l: [sph_begin[l], sph_begin[l+1])
  float4 sph[MAXS];              // local centre, radius
  float4 link_bs[MAXJ];          // link bounding sphere: local centre, radius (inflated); w < 0: none
  float4 point_sph;              // sphere family: offset and radius of the point robot
  float4 clus_lo[MAXC];          // cluster box: lower corner (xyz)
  float4 clus_hi[MAXC];          // cluster box: upper corner (xyz)
  int2 clus_range[MAXC];         // obstacle index range of each cluster
  float4 sup_lo[MAXSUP];         // group box: lower corner
  float4 sup_hi[MAXSUP];         // group box: upper corner
  int2 sup_range[MAXSUP];        // cluster index range of each group
};

// Squared distance from point c to the box [lo, hi] (0 inside).
// Resident waves per SIMD a model's FP32 stacked projection kernel is built for: a model (or its
// topology) may ask for 2 where the kernel fits in 256 registers per lane, so that twice the lanes
// run at once; 1 otherwise.
template <class M, class = void>
struct PersistWaves {
  static constexpr int value = 1;
};
template <class M>
struct PersistWaves<M, std::void_t<decltype(M::persist_waves)>> {
  static constexpr int value = M::persist_waves;
};

__device__ __forceinline__ float box_dist2(const float* c, const float4& lo, const float4& hi) {
  const float dx = fmaxf(fmaxf(lo.x - c[0], c[0] - hi.x), 0.f);
  const float dy = fmaxf(fmaxf(lo.y - c[1], c[1] - hi.y), 0.f);
  const float dz = fmaxf(fmaxf(lo.z - c[2], c[2] - hi.z), 0.f);
  return dx * dx + dy * dy + dz * dz;
}

struct DevProblem {
  Consts c;
  CollConsts k;
  const float4* obs;             // obstacles (x, y, z, r), grouped by cluster, n_obs of them
  unsigned long long* fallback_counter;
};

template <class T> __device__ __forceinline__ const TP<T>& tp(const Consts& P);
template <> __device__ __forceinline__ const TP<double>& tp<double>(const Consts& P) { return P.d; }
template <> __device__ __forceinline__ const TP<float>& tp<float>(const Consts& P) { return P.f; }

// Cooperative copy of `bytes` (multiple of 16) from global memory into LDS by the whole block.
__device__ __forceinline__ void block_copy16(void* dst_lds, const void* src, int bytes) {
  const uint4* s = static_cast<const uint4*>(src);
  uint4* d = static_cast<uint4*>(dst_lds);
  for (int i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

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

// Opaque copy: stops the compiler from proving two recomputations equal (and merging
// them, which would keep every intermediate live across the solve).
__device__ __forceinline__ float opaque(float x) { asm volatile("" : "+v"(x)); return x; }
__device__ __forceinline__ double opaque(double x) { asm volatile("" : "+v"(x)); return x; }
// Conversion of an FP64 result to the step precision S, pinned where it is written: the compiler
// would otherwise sink the conversion to the value's uses and keep the FP64 value (two registers)
// live through the kinematic walks in between.
template <class S>
__device__ __forceinline__ S to_step(double x) { return opaque(S(x)); }

// Ordering helper for the unrolled walks: an empty asm that claims to read `dep` and rewrite
// `x`, so x (and everything computed from it) cannot be scheduled before dep exists. Costs no
// instruction; bounds how far ahead loads and transcendental work are hoisted.
template <class T, class U>
__device__ __forceinline__ T after(T x, U dep) {
  asm volatile("" : "+v"(x) : "v"(dep));
  return x;
}
// Wave-uniform pointer, stated with readfirstlane so it can live in scalar registers.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
  return reinterpret_cast<T*>((uint64_t(hi) << 32) | lo);
}
// A reference into read-only global memory whose reads become scalar loads (constant address
// space), issued only after dep exists.
template <class T, class U>
__device__ __forceinline__ const T& after_const(const T& r, U dep) {
  using CT = const __attribute__((address_space(4))) T;
  CT* c = (CT*)uniform_ptr(&r);
  asm volatile("" : "+s"(c) : "v"(dep));
  return *(const T*)c;
}
// The problem's constants as scalar-load memory.
__device__ __forceinline__ const Consts& consts_of(const DevProblem* P) {
  using CT = const __attribute__((address_space(4))) Consts;
  CT* c = (CT*)uniform_ptr(&P->c);
  asm volatile("" : "+s"(c));
  return *(const Consts*)c;
}
// The collision data and obstacle array as scalar-load memory (wave-uniform reads).
__device__ __forceinline__ const CollConsts& coll_of(const DevProblem* P) {
  using CT = const __attribute__((address_space(4))) CollConsts;
  CT* c = (CT*)uniform_ptr(&P->k);
  asm volatile("" : "+s"(c));
  return *(const CollConsts*)c;
}
__device__ __forceinline__ const float4* obs_of(const DevProblem* P) {
  using PT = const float4* const __attribute__((address_space(4)));
  const float4* o = *(PT*)uniform_ptr(&P->obs);
  using OT = const __attribute__((address_space(4))) float4;
  OT* oc = (OT*)uniform_ptr(o);
  return (const float4*)oc;
}
// Same for a reference into LDS: its reads happen after dep.
template <class T, class U>
__device__ __forceinline__ const T& after_lds(const T& r, U dep) {
  using LT = const __attribute__((address_space(3))) T;
  LT* p = (LT*)&r;
  asm volatile("" : "+v"(p) : "v"(dep));
  return *(const T*)p;
}

// a * b + c with c wave-uniform (a scalar register pair), as one v_fma_f64. Written out because
// the compiler otherwise prefers v_fmac_f64, whose addend must first be copied into a vector
// register pair (two extra moves per Horner step).
__device__ __forceinline__ double fma_su(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// Polynomial coefficients of the FP64 elementary functions below, read with scalar loads at the
// point of use: as literals the compiler materialises them once outside the Newton loop and
// keeps them live (and spilled) across it.
struct alignas(16) MathTab {
  double sin_c[7];   // (-1)^k / (2k+1)!, k = 7 .. 1 (Horner order)
  double cos_c[8];   // (-1)^k / (2k)!, k = 8 .. 1
  double atan_c[14]; // (-1)^k / (2k+1), k = 14 .. 1
  double beta_c[5];  // series of 1/theta^2 - cot(theta/2)/(2 theta) in theta^2, highest first
};
static __constant__ MathTab kMathTab = {
    {-1.0 / 1307674368000.0, 1.0 / 6227020800.0, -1.0 / 39916800.0, 1.0 / 362880.0, -1.0 / 5040.0, 1.0 / 120.0,
     -1.0 / 6.0},
    {1.0 / 20922789888000.0, -1.0 / 87178291200.0, 1.0 / 479001600.0, -1.0 / 3628800.0, 1.0 / 40320.0, -1.0 / 720.0,
     1.0 / 24.0, -0.5},
    {-1.0 / 29.0, 1.0 / 27.0, -1.0 / 25.0, 1.0 / 23.0, -1.0 / 21.0, 1.0 / 19.0, -1.0 / 17.0, 1.0 / 15.0, -1.0 / 13.0,
     1.0 / 11.0, -1.0 / 9.0, 1.0 / 7.0, -1.0 / 5.0, 1.0 / 3.0},
    {1.0 / 47900160.0, 1.0 / 1209600.0, 1.0 / 30240.0, 1.0 / 720.0, 1.0 / 12.0},
};

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
  const MathTab& T = after_const(kMathTab, r2);
  double ps = T.sin_c[0];
  for (int i = 1; i < 7; ++i) ps = fma_su(ps, r2, T.sin_c[i]);
  const double sn = __builtin_fma(ps * r2, r, r);
  double pc = T.cos_c[0];
  for (int i = 1; i < 8; ++i) pc = fma_su(pc, r2, T.cos_c[i]);
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
__device__ __forceinline__ bool finite_t(double x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool finite_t(float x) { return __builtin_isfinite(x); }

// Accessors for the FP64 iterate. at(j) returns coordinate j; at(j, dep) reads it only after
// dep exists. Reads go through an opaque copy so separate passes never share them.
// Per-lane column of a wave's [D][64] FP64 tile in LDS: coordinate j at base[64 j], so every
// access is one ds_read/ds_write with an immediate offset (no per-coordinate address registers)
// and the 64 lanes of a wave hit 64 consecutive doubles.
struct QLds {
  using LP = __attribute__((address_space(3))) double*;
  LP base;
  __device__ __forceinline__ double at(int j) const { return opaque(base[j * 64]); }
  template <class U>
  __device__ __forceinline__ double at(int j, U dep) const {
    LP b = base;
    asm volatile("" : "+v"(b) : "v"(dep));
    return opaque(b[j * 64]);
  }
  __device__ __forceinline__ void set(int j, double v) const { base[j * 64] = v; }
  __device__ __forceinline__ double operator[](int j) const { return at(j); }
};
// One configuration shared by the 64 lanes of a wave (D consecutive doubles; every lane reads the
// same address, an LDS broadcast).
struct QLdsU {
  using LP = __attribute__((address_space(3))) double*;
  LP base;
  __device__ __forceinline__ double at(int j) const { return opaque(base[j]); }
  template <class U>
  __device__ __forceinline__ double at(int j, U dep) const {
    LP b = base;
    asm volatile("" : "+v"(b) : "v"(dep));
    return opaque(b[j]);
  }
  __device__ __forceinline__ void set(int j, double v) const { base[j] = v; }
};
// The calling lane's column; smem holds blockDim.x / 64 tiles of D x 64 doubles.
template <int D>
__device__ __forceinline__ QLds q_lds(double* smem) {
  const int w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  return QLds{(QLds::LP)(smem + w * (D * 64) + l)};
}
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
// C = A B
template <class T>
__device__ __forceinline__ void matmul3(const T* A, const T* B, T* C) {
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) C[3 * i + k] = A[3 * i] * B[k] + A[3 * i + 1] * B[3 + k] + A[3 * i + 2] * B[6 + k];
}

// atan2(y, x) on [0, pi] for y >= 0 (the rotation angle from sin and cos). Octant reduction to
// u = min/max in [0, 1], then u > tan(pi/12) is mapped to (u sqrt3 - 1) / (u + sqrt3) =
// tan(atan(u) - pi/6), so the Maclaurin series of atan runs on |u| <= tan(pi/12) = 0.268 and
// is truncated after u^29 / 29 (remainder below 1e-19).
__device__ __forceinline__ double angle_from_sincos(double y, double x) {
  const double ax = fabs(x);
  const double lo = fmin(y, ax), hi = fmax(y, ax);
  double u = lo / hi;
  const bool shift = u > 0.2679491924311228;
  u = shift ? (u * 1.7320508075688772 - 1.0) / (u + 1.7320508075688772) : u;
  const double u2 = u * u;
  const MathTab& T = after_const(kMathTab, u2);
  double p = T.atan_c[0];
  for (int i = 1; i < 14; ++i) p = fma_su(p, u2, T.atan_c[i]);
  double t = __builtin_fma(-p * u2, u, u);
  t = shift ? t + 0.5235987755982989 : t;          // + pi/6
  t = y > ax ? 1.5707963267948966 - t : t;        // pi/2 - t
  t = x < 0.0 ? 3.141592653589793 - t : t;        // pi - t
  return hi > 0.0 ? t : 0.0;
}

// SO(3) log (vee form) of R plus the left-Jacobian inverse J_l^-1(w), used for the angular
// rows of the pose errors (Eq. 1, Eq. 2): v = vee(R - R^T)/2 = sin(theta) * axis,
// c = cos(theta), w = (theta / sin theta) v, with the first-order Taylor form 1 + s^2/6 of
// theta / sin(theta) when sin^2(theta) < 1e-8 and theta < pi/2 (Sec. IV-A). For a left
// perturbation R' = exp([e]x) R, d log(R') / d e = J_l^-1(w) = I - [w]x / 2 + beta [w]x^2 with
// beta = 1/theta^2 - (1 + c) / (2 theta s), taken from its series when theta^2 < 0.1. Both
// forms of each factor are computed and selected, so lanes do not diverge.
__device__ __forceinline__ void so3_log_jlinv(const double* R, double* w, double* Jinv) {
  const double v0 = 0.5 * (R[7] - R[5]), v1 = 0.5 * (R[2] - R[6]), v2 = 0.5 * (R[3] - R[1]);
  const double s2 = v0 * v0 + v1 * v1 + v2 * v2;
  const double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
  const double sn = sqrt(s2);
  const double th = angle_from_sincos(sn, c);
  const bool small = c > 0.0 && s2 < 1e-8;
  const double f = small ? __builtin_fma(s2, 1.0 / 6.0, 1.0) : th / sn;
  w[0] = f * v0; w[1] = f * v1; w[2] = f * v2;
  if (Jinv) {
    const double th2 = f * f * s2;
    // 1/theta^2 - cot(theta/2) / (2 theta) = 1/12 + th^2/720 + th^4/30240 + th^6/1209600 + th^8/47900160 + ...
    const MathTab& T = after_const(kMathTab, th2);
    double bs = T.beta_c[0];
    for (int i = 1; i < 5; ++i) bs = fma_su(bs, th2, T.beta_c[i]);
    const double bc = 1.0 / th2 - (1.0 + c) / (2.0 * th * sn);
    const double beta = th2 < 0.1 ? bs : bc;
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
