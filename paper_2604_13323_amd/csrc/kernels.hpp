// Generic HIP kernels of the projection path, templated on the constraint model.
//
// Mapping: one configuration per lane; the lane's FP64 iterate lives in LDS (a column
// of a [D][blockDim] array, conflict-free); the kinematic constants are read with scalar
// loads (wave-uniform, so they occupy scalar registers), the collision data is staged in
// LDS once per workgroup; everything else is in registers. The hot
// loop (Alg. 2 ParallelProject with getDescentStep on one stacked block) per iteration:
//   1. residual pass, FP64: forward kinematics, F(q), ||F||^2, and the per-block data
//      the Jacobian columns need;
//   2. convergence test ||F||^2 < tol^2 (per lane; a wave leaves the loop when every
//      lane is done);
//   3. Gram pass in the step precision: forward kinematics again, each Jacobian column
//      is formed and folded into J J^T (structural nonzeros only); J is never stored;
//   4. in-register Cholesky of J J^T (+ lambda I) with the condition estimate
//      (max L_ii / min L_ii)^2 and forward/back substitution for y = (J J^T)^-1 F;
//      lanes whose estimate exceeds the threshold, or whose factorisation fails,
//      redo 1, 3 and 4 in FP64;
//   5. J^T y pass (forward kinematics a third time), dq = alpha J^T y, optional
//      divergence exit, q <- q - dq.
// The persistent variant refills a lane from a device work queue as soon as its
// configuration finishes, so lanes do not idle until the slowest configuration of
// their wave converges.
#pragma once

#include "common.hpp"

namespace mc {

struct ProjArgs {
  const DevProblem* P;
  int64_t n;          // configurations handled by this launch
  int64_t base;       // index of the first one in the caller's arrays
  const void* q_in;
  int64_t ld_in;
  void* q_out;
  int64_t ld_out;
  int8_t* status;
  int8_t* iters;
  void* resid;
  uint8_t* verdict;   // plain fused kernel only
  double tol2, alpha, lambda, max_step, cond_thr;
  int32_t max_iter;
  int32_t check;
  int32_t outer;          // 1: the outer form of the step, (J^T J + lambda I)^-1 J^T F (families with D <= kOuterMaxD)
  unsigned int* counter;  // persistent: queue head (reset to 0 before the launch)
  int64_t n_static;       // persistent: configurations [0, n_static) are taken by thread id
  // FP32 mode: configurations whose FP32 step fails (factorisation or condition estimate) are
  // handed to the FP64 tail kernel through this queue: defer_ik[2s], defer_ik[2s+1] = index and
  // steps taken, defer_q[c * defer_cap + s] = FP64 iterate.
  unsigned int* defer_count;
  int32_t* defer_ik;
  double* defer_q;
  int64_t defer_cap;
  // Fused collision check: converged configurations whose broad-phase test found a link near
  // the obstacles are queued here for the exact check
  // (index in chk_idx[s], FP64 configuration at chk_q[c * defer_cap + s]).
  unsigned int* chk_count;
  int32_t* chk_idx;
  double* chk_q;
  int32_t n_sph, n_obs;   // robot and obstacle spheres (LDS size of the exact-check kernel)
  int32_t chk_lanes;      // exact-check tail: lanes per queued configuration (0: by queue length; 1, 2, 4, 8, 16, 64)
  int32_t chk_long;       // exact-check tail: lanes per configuration on a long queue with chk_lanes = 0
                          // (1, 2, 4, 8 or 16; 0 = kTailCheckLanesLong)
};

constexpr int ST_DEFER = -2;  // internal: continue this configuration with FP64 steps

template <class IO>
__device__ __forceinline__ double ld_io(const void* p, int64_t k) { return double(static_cast<const IO*>(p)[k]); }
template <class IO>
__device__ __forceinline__ void st_io(void* p, int64_t k, double v) { static_cast<IO*>(p)[k] = IO(v); }

template <class IO>
struct QGlob {  // configuration i of a [D][ld] array in global memory
  const IO* p;
  int64_t ld, i;
  int dof;
  __device__ __forceinline__ double at(int j) const { return j < dof ? double(p[j * ld + i]) : 0.0; }
  template <class U>
  __device__ __forceinline__ double at(int j, U) const { return at(j); }
};

// ------------------------------------------------------------------ Cholesky
// Rows a lane has dropped (bits of Model::DROPPABLE; none for models that never drop rows).
template <class Model, class SDT>
__device__ __forceinline__ uint32_t drop_bits(const SDT& sd) {
  if constexpr (Model::DROPPABLE != 0) return sd.drop;
  else return 0u;
}

// In-place right-looking Cholesky of the packed lower triangle G (structural zeros of the
// factor skipped at compile time). Returns false on a non-positive or non-finite pivot, or a
// pivot below floor. invd receives 1 / L_ii; kappa the estimate (max L_ii / min L_ii)^2.
// A dropped row (its G row and column are zero) gets the unit pivot and takes no part in kappa.
template <class Model, class S, uint32_t RM = ~uint32_t(0)>
__device__ __forceinline__ bool cholesky(S* G, S* invd, S& kappa, S floor, uint32_t drop = 0u) {
  constexpr int M = Model::M;
  bool ok = true;
  S dmin = S(3.0e38), dmax = S(0);
  sfor<0, M>([&](auto K) {
    constexpr int k = decltype(K)::value;
    if constexpr (((RM >> k) & 1u) != 0) {
    bool dk = false;
    if constexpr (((Model::DROPPABLE >> k) & 1u) != 0) dk = ((drop >> k) & 1u) != 0;
    const S d = dk ? S(1) : G[pidx(k, k)];
    ok = ok && (dk || ((d > floor) && finite_t(d)));
    const S r = rsqrt_t(d);
    const S l = d * r;
    G[pidx(k, k)] = l;
    invd[k] = r;
    dmin = (dk || !(l < dmin)) ? dmin : l;
    dmax = (dk || !(l > dmax)) ? dmax : l;
    sfor<k + 1, M>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (Model::lnz(i, k) && ((RM >> i) & 1u)) G[pidx(i, k)] *= r;
    });
    sfor<k + 1, M>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (Model::lnz(i, k) && ((RM >> i) & 1u)) {
        sfor<k + 1, i + 1>([&](auto Jx) {
          constexpr int j = decltype(Jx)::value;
          if constexpr (Model::lnz(j, k) && ((RM >> j) & 1u)) G[pidx(i, j)] -= G[pidx(i, k)] * G[pidx(j, k)];
        });
      }
    });
    }
  });
  S ratio = dmax / dmin;
  if constexpr (Model::DROPPABLE != 0) ratio = dmax > S(0) ? ratio : S(0);  // every row dropped
  kappa = ratio * ratio;
  return ok && finite_t(kappa);
}

// Solve L L^T y = b in place (b overwritten by y).
template <class Model, class S, uint32_t RM = ~uint32_t(0)>
__device__ __forceinline__ void chol_solve(const S* L, const S* invd, S* y) {
  constexpr int M = Model::M;
  sfor<0, M>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr ((RM >> i) & 1u) {
      S acc = y[i];
      sfor<0, i>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (Model::lnz(i, k) && ((RM >> k) & 1u)) acc -= L[pidx(i, k)] * y[k];
      });
      y[i] = acc * invd[i];
    }
  });
  sfor<0, M>([&](auto I) {
    constexpr int i = M - 1 - decltype(I)::value;
    if constexpr ((RM >> i) & 1u) {
      S acc = y[i];
      sfor<i + 1, M>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (Model::lnz(k, i) && ((RM >> k) & 1u)) acc -= L[pidx(k, i)] * y[k];
      });
      y[i] = acc * invd[i];
    }
  });
}

constexpr float kFloorF32 = 0.0f;
constexpr double kFloorF64 = 1e-24;  // pivot floor relative to the largest Gram diagonal entry

// One descent step in precision S: dq = J^T (J J^T + lambda I)^-1 rhs (rhs = F for Newton;
// overwritten). Returns false when the factorisation fails or its condition estimate
// exceeds cond_thr.
// RM restricts the system to the rows of one block (cyclic mode).
template <class Model, class S, uint32_t RM = ~uint32_t(0), class Q>
__device__ __forceinline__ bool descent_step(const Q& q, S* rhs, const typename Model::template SD<S>& sd,
                                             const Consts& C, double lambda, double cond_thr, S floor_rel, S* dq) {
  constexpr int M = Model::M;
  S G[M * (M + 1) / 2];
  Model::template gram<S, false, RM>(q, C, sd, G, nullptr, nullptr);
  S maxd = S(0);
  sfor<0, M>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr ((RM >> i) & 1u) {
      G[pidx(i, i)] += S(lambda);
      maxd = G[pidx(i, i)] > maxd ? G[pidx(i, i)] : maxd;
    }
  });
  S invd[M], kappa;
  if (!cholesky<Model, S, RM>(G, invd, kappa, floor_rel * maxd, drop_bits<Model>(sd))) return false;
  if (!(double(kappa) <= cond_thr)) return false;
  chol_solve<Model, S, RM>(G, invd, rhs);
  Model::template jty<S, RM>(q, C, sd, rhs, dq);
  return true;
}

// ------------------------------------------------------------------ outer form of the step
// The step's alternative form (Alg. 2 getDescentStep; Sec. IV-A provides the inner and the outer
// pseudo-inverse): dq = (J^T J + lambda I)^-1 J^T F, a d x d system, for lambda > 0. Built for the
// families with d <= kOuterMaxD, whose dense J and packed d x d factor fit a lane's registers.
constexpr int kOuterMaxD = 16;

// Dense packed-lower Cholesky of an N x N matrix in place (all entries), with the same conventions
// as cholesky(): false on a pivot <= floor or non-finite; invd = 1 / L_ii; kappa = (max / min L_ii)^2.
template <int N, class S>
__device__ __forceinline__ bool dense_cholesky(S* A, S* invd, S& kappa, S floor) {
  bool ok = true;
  S dmin = S(3.0e38), dmax = S(0);
  sfor<0, N>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const S d = A[pidx(k, k)];
    ok = ok && (d > floor) && finite_t(d);
    const S r = rsqrt_t(d);
    const S l = d * r;
    A[pidx(k, k)] = l;
    invd[k] = r;
    dmin = l < dmin ? l : dmin;
    dmax = l > dmax ? l : dmax;
    sfor<k + 1, N>([&](auto I) { A[pidx(decltype(I)::value, k)] *= r; });
    sfor<k + 1, N>([&](auto I) {
      constexpr int i = decltype(I)::value;
      sfor<k + 1, i + 1>([&](auto Jx) {
        constexpr int j = decltype(Jx)::value;
        A[pidx(i, j)] -= A[pidx(i, k)] * A[pidx(j, k)];
      });
    });
  });
  const S ratio = dmax / dmin;
  kappa = ratio * ratio;
  return ok && finite_t(kappa);
}

template <int N, class S>
__device__ __forceinline__ void dense_solve(const S* L, const S* invd, S* y) {
  sfor<0, N>([&](auto I) {
    constexpr int i = decltype(I)::value;
    S acc = y[i];
    sfor<0, i>([&](auto K) { acc -= L[pidx(i, decltype(K)::value)] * y[decltype(K)::value]; });
    y[i] = acc * invd[i];
  });
  sfor<0, N>([&](auto I) {
    constexpr int i = N - 1 - decltype(I)::value;
    S acc = y[i];
    sfor<i + 1, N>([&](auto K) { acc -= L[pidx(decltype(K)::value, i)] * y[decltype(K)::value]; });
    y[i] = acc * invd[i];
  });
}

// dq = (J^T J + lambda I)^-1 J^T rhs with the dense Jacobian of the step pass (dropped rows are zero
// rows of J and need no special case: lambda > 0 keeps the d x d matrix positive definite).
template <class Model, class S, class Q>
__device__ __forceinline__ bool descent_step_outer(const Q& q, const S* rhs, const typename Model::template SD<S>& sd,
                                                   const Consts& C, double lambda, double cond_thr, S floor_rel, S* dq) {
  constexpr int D = Model::D, M = Model::M;
  S J[M * D];
  Model::template jacobian<S>(q, C, sd, J);
  S A[D * (D + 1) / 2];
  S maxd = S(0);
  sfor<0, D>([&](auto I) {
    constexpr int i = decltype(I)::value;
    sfor<0, i + 1>([&](auto K) {
      constexpr int k = decltype(K)::value;
      S acc = (i == k) ? S(lambda) : S(0);
      for (int r = 0; r < M; ++r) acc += J[r * D + i] * J[r * D + k];
      A[pidx(i, k)] = acc;
    });
    maxd = A[pidx(i, i)] > maxd ? A[pidx(i, i)] : maxd;
    S b = S(0);
    for (int r = 0; r < M; ++r) b += J[r * D + i] * rhs[r];
    dq[i] = b;
  });
  S invd[D], kappa;
  if (!dense_cholesky<D, S>(A, invd, kappa, floor_rel * maxd)) return false;
  if (!(double(kappa) <= cond_thr)) return false;
  dense_solve<D, S>(A, invd, dq);
  return true;
}

// The step in the form the call asked for.
template <class Model, class S, class Q>
__device__ __forceinline__ bool step_of(const Q& q, S* rhs, const typename Model::template SD<S>& sd, const Consts& C,
                                        const ProjArgs& a, double cond_thr, S floor_rel, S* dq) {
  if constexpr (Model::D <= kOuterMaxD) {
    if (a.outer) return descent_step_outer<Model, S>(q, rhs, sd, C, a.lambda, cond_thr, floor_rel, dq);
  }
  return descent_step<Model, S>(q, rhs, sd, C, a.lambda, cond_thr, floor_rel, dq);
}

// Apply dq (scaled by alpha) with the divergence test. Returns -1 after the update or a status.
template <class Model, class S>
__device__ __forceinline__ int apply_step(const QLds& q, const S* dq, const ProjArgs& a) {
  constexpr int D = Model::D;
  double s2 = 0.0;
  for (int j = 0; j < D; ++j) {
    const double d = a.alpha * double(dq[j]);
    s2 += d * d;
  }
  if (!finite_t(s2)) return ST_NONFINITE;
  if (a.max_step > 0.0 && s2 > a.max_step * a.max_step) return ST_DIVERGED;
  for (int j = 0; j < D; ++j) q.set(j, q.at(j) - a.alpha * double(dq[j]));
  return -1;
}

// One Newton iteration for one lane: residual and convergence test in FP64, then the step in
// precision S. Returns -1 after taking a step, else the final status; in FP32 mode ST_DEFER
// when the FP32 factorisation fails or its condition estimate exceeds the threshold (the
// iteration is then redone with an FP64 step, and the configuration stays in FP64 until it
// ends).
template <class Model, class S>
__device__ __forceinline__ int newton_iteration(const QLds& q, int& k, const ProjArgs& a, const Consts& C, double& resid) {
  constexpr int D = Model::D, M = Model::M;
  typename Model::template SD<S> sd;
  S F[M];
  const double n2 = Model::template residual<S>(q, C, F, sd);
  resid = sqrt(n2);
  if (!finite_t(n2)) return ST_NONFINITE;
  if (n2 < a.tol2) return ST_CONVERGED;
  if (k >= a.max_iter) return ST_MAX_ITER;
  S dq[D];
  int st;
  if constexpr (std::is_same<S, float>::value) {
    if (!step_of<Model, float>(q, F, sd, C, a, a.cond_thr, kFloorF32, dq)) return ST_DEFER;
    st = apply_step<Model, float>(q, dq, a);
  } else {
    if (!step_of<Model, double>(q, F, sd, C, a, 1e300, kFloorF64, dq)) return ST_SINGULAR;
    st = apply_step<Model, double>(q, dq, a);
  }
  if (st < 0) ++k;
  return st;
}

// One iteration of the cyclic mode (Alg. 2, getDescentStep looping over the constraints, Sec.
// IV-C): the full residual and the convergence test, then one min-norm step per constraint block
// in order, each taken from the configuration the previous block left; the divergence test
// (MaxDistance) applies to the displacement of the whole iteration. q0 receives the iterate at
// the start of the iteration. In FP32 mode a failed factorisation in any block restores that
// iterate and returns ST_DEFER (the iteration is redone in FP64).
template <class Model, class S>
__device__ __forceinline__ int cyclic_iteration(const QLds& q, const QLds& q0, int& k, const ProjArgs& a,
                                                const Consts& C, double& resid) {
  constexpr int D = Model::D, M = Model::M, NB = Model::NBLK;
  constexpr bool f32 = std::is_same<S, float>::value;
  typename Model::template SD<S> sd;
  S F[M];
  const double n2 = Model::template residual<S>(q, C, F, sd);
  resid = sqrt(n2);
  if (!finite_t(n2)) return ST_NONFINITE;
  if (n2 < a.tol2) return ST_CONVERGED;
  if (k >= a.max_iter) return ST_MAX_ITER;
  for (int c = 0; c < D; ++c) q0.set(c, q.at(c));
  int st = -1;
  bool failed = false;
  sfor<0, NB>([&](auto BI) {
    constexpr int b = decltype(BI)::value;
    constexpr uint32_t RM = Model::block_rows_mask(b);
    if (st < 0 && !failed) {
      // the first block steps from the iterate whose residual is already in F and sd
      if constexpr (b > 0) Model::template residual<S, RM>(q, C, F, sd);
      S dq[D];
      if (!descent_step<Model, S, RM>(q, F, sd, C, a.lambda, f32 ? a.cond_thr : 1e300, f32 ? S(kFloorF32) : S(kFloorF64),
                                      dq)) {
        failed = true;
      } else {
        double s2 = 0.0;
        for (int j = 0; j < D; ++j) {
          const double dj = a.alpha * double(dq[j]);
          s2 += dj * dj;
        }
        if (!finite_t(s2)) st = ST_NONFINITE;
        else
          for (int j = 0; j < D; ++j) q.set(j, q.at(j) - a.alpha * double(dq[j]));
      }
    }
  });
  if (failed) {
    if constexpr (f32) {
      for (int c = 0; c < D; ++c) q.set(c, q0.at(c));
      return ST_DEFER;
    } else {
      return ST_SINGULAR;
    }
  }
  if (st >= 0) return st;
  if (a.max_step > 0.0) {
    double s2 = 0.0;
    for (int c = 0; c < D; ++c) {
      const double t = q.at(c) - q0.at(c);
      s2 += t * t;
    }
    if (s2 > a.max_step * a.max_step) {
      for (int c = 0; c < D; ++c) q.set(c, q0.at(c));
      return ST_DIVERGED;
    }
  }
  ++k;
  return -1;
}

// One iteration of either mode.
template <class Model, class S, bool CYC>
__device__ __forceinline__ int iteration(const QLds& q, const QLds& q0, int& k, const ProjArgs& a, const Consts& C,
                                         double& resid) {
  if constexpr (CYC) return cyclic_iteration<Model, S>(q, q0, k, a, C, resid);
  else return newton_iteration<Model, S>(q, k, a, C, resid);
}

// Run one configuration to the end with FP64 steps.
template <class Model, bool CYC = false>
__device__ __forceinline__ int finish_fp64(const QLds& q, const QLds& q0, int& k, const ProjArgs& a, const Consts& C,
                                          double& resid) {
  int st;
  do {
    st = iteration<Model, double, CYC>(q, q0, k, a, C, resid);
  } while (st < 0);
  return st;
}

// Configuration dimension: a compile-time constant where the model fixes it (the per-coordinate
// guards of the load and store loops then fold away), else the scene's value.
template <class Model>
__device__ __forceinline__ int dof_of(const Consts& C) {
  if constexpr (Model::fixed_dof) return Model::D;
  else return C.dof;
}

// Column c of configuration i in a [D][ld] array sits at (c ld + i); the pointer is bumped by
// an opaque ld so the D addresses are formed one after another rather than all up front.
template <class Model, class IO>
__device__ __forceinline__ void load_q(const ProjArgs& a, int dof, int64_t i, const QLds& q) {
  const IO* p = static_cast<const IO*>(a.q_in) + a.base + i;
  const int64_t ld = a.ld_in;
  for (int c = 0; c < Model::D; ++c) {
    q.set(c, c < dof ? double(*p) : 0.0);
    p += after(ld, c);
  }
}

template <class Model, class IO>
__device__ __forceinline__ void store_result(const ProjArgs& a, int dof, int64_t i, const QLds& q, int st, int k,
                                             double resid) {
  IO* p = static_cast<IO*>(a.q_out) + a.base + i;
  const int64_t ld = a.ld_out;
  for (int c = 0; c < Model::D; ++c) {
    if (c < dof) *p = IO(q.at(c));
    p += after(ld, c);
  }
  a.status[a.base + i] = int8_t(st);
  a.iters[a.base + i] = int8_t(k);
  st_io<IO>(a.resid, a.base + i, resid);
}

// Persistent projection kernel: a grid of resident waves pulls configurations from a device
// work queue (atomic counter), one per lane, and refills a lane when its configuration ends.
// Dynamic LDS: D * blockDim doubles.
// Append the calling lane's FP64 configuration to a queue (slot < defer_cap: the queues are
// sized for the batch).
template <class Model, class Q>
__device__ __forceinline__ unsigned queue_q(const Q& q, unsigned* count, double* qbuf, int64_t cap) {
  const unsigned slot = atomicAdd(count, 1u);
  double* dst = qbuf + slot;
  for (int c = 0; c < Model::D; ++c) {
    *dst = q.at(c);
    dst += after(cap, c);
  }
  return slot;
}

template <class Model, class IO, class Q>
__device__ __forceinline__ void load_queued(const double* qbuf, int64_t cap, int64_t slot, const Q& q) {
  const double* src = qbuf + slot;
  for (int c = 0; c < Model::D; ++c) {
    q.set(c, *src);
    src += after(cap, c);
  }
}

// Collision verdict of a configuration that ended with status st (exact check in-line).
template <class Model>
__device__ __forceinline__ uint8_t verdict_inline(const QLds& q, const Consts& C, const ProjArgs& a, int st) {
  if (!a.check || st != ST_CONVERGED) return V_UNCHECKED;
  const CollConsts& K = coll_of(a.P);
  return Model::template check_group<1>(q, C, K, K.sph, obs_of(a.P)) ? V_HIT : V_FREE;
}

// Persistent projection kernel: a grid of resident waves pulls configurations from a device
// work queue (atomic counter), one per lane, and refills a lane when its configuration ends.
// With a verdict array the collision check is fused: tree models walk the converged
// configuration's link bounds once more in FP32 and test them against the box around the
// obstacles, so a configuration with no link near the obstacles is FREE at once, and the others
// are queued for the exact check (k_check_tail).
// Dynamic LDS: D * blockDim doubles.
template <class Model, class IO, class S, bool CYC>
__device__ __forceinline__ void persistent_body(const ProjArgs& a, double* smem) {
  const Consts& C = consts_of(a.P);
  const int dof = dof_of<Model>(C);
  const QLds q = q_lds<Model::D>(smem);
  const QLds q0 = q_lds<Model::D>(smem + (CYC ? Model::D * blockDim.x : 0));  // cyclic: iterate at iteration start
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n_static) i = a.n;  // not part of the static share
  int k = 0;
  if (i < a.n) load_q<Model, IO>(a, dof, i, q);
  constexpr bool fused = Model::broad_in_residual;
  // A converged lane that needs the broad phase waits (pending) until no lane of the wave is
  // still iterating or half the wave is waiting, so one FP32 walk serves all of them instead of
  // one walk per iteration count.
  bool pending = false;
  for (;;) {
    const bool active = i < a.n && !pending;
    const bool any_active = __any(active);
    if (!any_active && !__any(pending)) break;
    if (fused && (!any_active || __builtin_popcountll(uint64_t(__ballot(pending))) >= 32)) {
      if (pending) {
        // broad phase on the converged configurations (an FP32 walk of the link bounds)
        a.verdict[i] = V_FREE;  // k_check_tail overwrites it with V_HIT if some part finds a hit
        if (Model::broad_flag(q, C)) a.chk_idx[queue_q<Model>(q, a.chk_count, a.chk_q, a.defer_cap)] = int32_t(i);
        pending = false;
        i = a.n_static + int64_t(atomicAdd(a.counter, 1u));
        k = 0;
        if (i < a.n) load_q<Model, IO>(a, dof, i, q);
      }
      continue;
    }
    if (active) {
      double resid;
      int st = iteration<Model, S, CYC>(q, q0, k, a, C, resid);
      if (st == ST_DEFER) {
        const unsigned slot = queue_q<Model>(q, a.defer_count, a.defer_q, a.defer_cap);
        atomicAdd(a.P->fallback_counter, 1ull);
        a.defer_ik[2 * slot] = int32_t(i);
        a.defer_ik[2 * slot + 1] = k;
      } else if (st >= 0) {
        store_result<Model, IO>(a, dof, i, q, st, k, resid);
        if (a.verdict) {
          if constexpr (fused) {
            if (a.check && st == ST_CONVERGED) pending = true;  // the verdict comes with the wave's walk
            else a.verdict[i] = V_UNCHECKED;
          } else {
            a.verdict[i] = verdict_inline<Model>(q, C, a, st);
          }
        }
      }
      if ((st >= 0 || st == ST_DEFER) && !pending) {
        i = a.n_static + int64_t(atomicAdd(a.counter, 1u));
        k = 0;
        if (i < a.n) load_q<Model, IO>(a, dof, i, q);
      }
    }
  }
}


template <class Model, class S, bool CYC>
constexpr int persist_waves_v = std::is_same<S, float>::value && !CYC ? PersistWaves<Model>::value : 1;

template <class Model, class IO, class S, bool CYC = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(persist_waves_v<Model, S, CYC>)))
k_project_persistent(ProjArgs a) {
  extern __shared__ double smem[];
  persistent_body<Model, IO, S, CYC>(a, smem);
}

// The same kernel compiled for two resident waves per SIMD (registers capped at 256 per lane, the
// rest spilled): for batches larger than the lanes one wave per SIMD offers, where a second
// round of the work queue would otherwise run with nothing to hide its latency.
template <class Model, class IO, class S>
__global__ void __launch_bounds__(256, 2) k_project_persistent_wide(ProjArgs a) {
  extern __shared__ double smem[];
  persistent_body<Model, IO, S, false>(a, smem);
}

// Exact collision check of the configurations queued by k_project_persistent, L lanes per
// configuration (grid-stride over the queue). A short queue (at most `small` entries: latency-bound,
// few waves) runs a wave per configuration, each configuration's links split over up to 4 waves; a
// longer one runs groups of chk_long lanes (the autotuner's choice among 1, 2, 4, 8 and 16; 4 by
// default). Every lane of a group walks the tree, and the group splits the sphere-obstacle tests of
// the (link, cluster) pairs it finds overlapping: smaller groups repeat fewer walks, but the lanes of
// a wave then run different pair lists and the wave runs their union, so the best size depends on
// the batch. A caller may force 1, 2, 4, 8, 16 or 64 lanes (chk_lanes).
// Dynamic LDS: one configuration per lane group (D doubles each; a wave per configuration also
// keeps 64 candidate-sphere slots per wave), then the robot spheres and the obstacles (float4
// each); groups below 4 lanes exist for families of at most kTailCheckLowLanesMaxD
// coordinates and run only where their staged configurations leave room for 4 workgroups per CU
// (min_lanes, from the launcher).
constexpr int kTailCheckLanesLong = 4;
constexpr int kTailCheckLowLanesMaxD = 16;
constexpr size_t kTailCheckLdsBudget = 40 * 1024;  // a quarter of a CU's LDS

template <class Model, class IO, int L>
__device__ __forceinline__ void check_tail_body(const ProjArgs& a, int64_t small, int64_t cnt, double* smem) {
  constexpr int D = Model::D;
  const Consts& C = consts_of(a.P);
  const CollConsts& K = coll_of(a.P);
  int64_t parts = 1;
  if (L == 64 && cnt > 0) parts = small / cnt < 4 ? (small / cnt < 1 ? 1 : small / cnt) : 4;
  if (int64_t(blockIdx.x) * blockDim.x / L >= cnt * parts) return;  // no queued work for this block
  const QLdsU q{(QLdsU::LP)(smem + (threadIdx.x / L) * D)};
  // a wave per configuration: 64 candidate-sphere slots per wave after the configurations
  float4* slots = L == 64 ? reinterpret_cast<float4*>(smem + D * (blockDim.x / L)) + (threadIdx.x / 64) * 64 : nullptr;
  float4* sph = reinterpret_cast<float4*>(smem + D * (blockDim.x / L)) + (L == 64 ? (blockDim.x / 64) * 64 : 0);
  float4* obs = sph + K.n_sph;
  block_copy16(sph, K.sph, K.n_sph * 16);
  block_copy16(obs, obs_of(a.P), K.n_obs * 16);
  __syncthreads();
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t item = gid / L; item < cnt * parts; item += int64_t(gridDim.x) * blockDim.x / L) {
    const int64_t slot = item / parts;
    const int part = int(item - slot * parts);
    load_queued<Model, IO>(a.chk_q, a.defer_cap, slot, q);
    const bool hit = Model::template check_group<L>(q, C, K, sph, obs, part, int(parts), slots);
    if ((gid & (L - 1)) == 0 && hit) a.verdict[a.chk_idx[slot]] = V_HIT;  // queued as V_FREE
  }
}

template <class Model, class IO>
__global__ void __launch_bounds__(256) k_check_tail(ProjArgs a, int64_t small, int min_lanes) {
  extern __shared__ double smem[];
  const int64_t cnt = *a.chk_count;
  int L = a.chk_lanes != 0 ? a.chk_lanes : cnt <= small ? 64 : a.chk_long > 0 ? a.chk_long : kTailCheckLanesLong;
  if (L < min_lanes) L = min_lanes;
  if (L == 64) {
    check_tail_body<Model, IO, 64>(a, small, cnt, smem);
  } else if (L == 16) {
    check_tail_body<Model, IO, 16>(a, small, cnt, smem);
  } else if (L == 8) {
    check_tail_body<Model, IO, 8>(a, small, cnt, smem);
  } else if constexpr (Model::D <= kTailCheckLowLanesMaxD) {
    if (L == 1) check_tail_body<Model, IO, 1>(a, small, cnt, smem);
    else if (L == 2) check_tail_body<Model, IO, 2>(a, small, cnt, smem);
    else check_tail_body<Model, IO, 4>(a, small, cnt, smem);
  } else {
    check_tail_body<Model, IO, 4>(a, small, cnt, smem);
  }
}

// FP64 tail of the persistent variant: the configurations deferred by the FP32 kernel, one per
// lane (grid-stride over the queue), continued from their stored FP64 iterate with FP64 steps. Their
// collision check joins the persistent kernel's: broad phase here, flagged ones queued for
// k_check_tail (a one-lane exact check in-line cost C1's tail half a millisecond).
// Dynamic LDS: D * blockDim doubles.
template <class Model, class IO, bool CYC = false>
__global__ void __launch_bounds__(64) k_project_tail(ProjArgs a) {
  extern __shared__ double smem[];
  const Consts& C = consts_of(a.P);
  const int dof = dof_of<Model>(C);
  const QLds q = q_lds<Model::D>(smem);
  const QLds q0 = q_lds<Model::D>(smem + (CYC ? Model::D * blockDim.x : 0));
  const int64_t cnt = *a.defer_count;
  for (int64_t slot = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; slot < cnt;
       slot += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = a.defer_ik[2 * slot];
    int k = a.defer_ik[2 * slot + 1];
    load_queued<Model, IO>(a.defer_q, a.defer_cap, slot, q);
    double resid;
    const int st = finish_fp64<Model, CYC>(q, q0, k, a, C, resid);
    store_result<Model, IO>(a, dof, i, q, st, k, resid);
    if (a.verdict) {
      if constexpr (Model::broad_in_residual) {
        // as in the persistent kernel: the broad phase here, the exact check of flagged
        // configurations in k_check_tail (launched after this kernel), with its lane groups
        if (a.check && st == ST_CONVERGED) {
          a.verdict[i] = V_FREE;
          if (Model::broad_flag(q, C)) a.chk_idx[queue_q<Model>(q, a.chk_count, a.chk_q, a.defer_cap)] = int32_t(i);
        } else {
          a.verdict[i] = V_UNCHECKED;
        }
      } else {
        a.verdict[i] = verdict_inline<Model>(q, C, a, st);
      }
    }
  }
}

// Plain kernel: one launch per geodesic, one configuration per lane, projection and
// collision check in the same kernel, no work queues (the FP64 steps and the exact check of
// flagged configurations run in-line).
template <class Model, class IO, class S>
__global__ void __launch_bounds__(64) k_project_plain(ProjArgs a) {
  extern __shared__ double smem[];
  const Consts& C = consts_of(a.P);
  const int dof = dof_of<Model>(C);
  const QLds q = q_lds<Model::D>(smem);
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  load_q<Model, IO>(a, dof, i, q);
  int k = 0, st;
  double resid;
  constexpr bool fused = Model::broad_in_residual;
  bool near = true;
  for (;;) {
    st = newton_iteration<Model, S>(q, k, a, C, resid);
    if (st >= 0) break;
    if (st == ST_DEFER) {  // same rule as the persistent variant: FP64 steps from here on
      atomicAdd(a.P->fallback_counter, 1ull);
      st = finish_fp64<Model>(q, q, k, a, C, resid);
      near = true;
      break;
    }
  }
  store_result<Model, IO>(a, dof, i, q, st, k, resid);
  if (a.verdict) {
    // same broad-phase rule as the persistent variant; the exact check runs in-line
    if (fused && a.check && st == ST_CONVERGED) near = Model::broad_flag(q, C);
    const bool skip = fused && a.check && st == ST_CONVERGED && !near;
    a.verdict[a.base + i] = skip ? uint8_t(V_FREE) : verdict_inline<Model>(q, C, a, st);
  }
}

struct CheckArgs {
  const DevProblem* P;
  int64_t n;
  const void* q;
  int64_t ld;
  const int8_t* status;  // nullable: check only CONVERGED configurations
  uint8_t* verdict;
  void* minsd;           // nullable
};

// check_batch: L lanes per configuration (L = 1 with the exhaustive minimum signed distance).
template <class Model, class IO, bool MINSD, int L>
__global__ void __launch_bounds__(256) k_check(CheckArgs a) {
  const Consts& C = consts_of(a.P);
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t i = gid / L;
  if (i >= a.n) return;  // whole groups leave together
  const bool lead = (gid & (L - 1)) == 0;
  if (a.status && a.status[i] != ST_CONVERGED) {
    if (lead) a.verdict[i] = V_UNCHECKED;
    return;
  }
  const QGlob<IO> q{static_cast<const IO*>(a.q), a.ld, i, dof_of<Model>(C)};
  if constexpr (MINSD) {
    static_assert(L == 1, "the exhaustive distance runs one lane per configuration");
    bool hit;
    float msd;
    Model::min_signed_distance(q, C, coll_of(a.P), obs_of(a.P), hit, msd);
    a.verdict[i] = hit ? V_HIT : V_FREE;
    st_io<IO>(a.minsd, i, double(msd));
  } else {
    const CollConsts& K = coll_of(a.P);
    const bool hit = Model::template check_group<L>(q, C, K, K.sph, obs_of(a.P));
    if (lead) a.verdict[i] = hit ? V_HIT : V_FREE;
  }
}

// check_batch without distances, first pass: one lane per configuration, the FP32 walk of the link
// bounds against the box around all obstacles (the same broad phase as the fused projection). A
// configuration with no link near the box is FREE; the others are marked FREE and queued (index,
// FP64 configuration) for k_check_tail, which overwrites the verdict of those it finds colliding.
template <class Model, class IO>
__global__ void __launch_bounds__(256) k_check_broad(CheckArgs a, unsigned* count, int32_t* idx, double* qbuf,
                                                     int64_t cap) {
  const Consts& C = consts_of(a.P);
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  if (a.status && a.status[i] != ST_CONVERGED) {
    a.verdict[i] = V_UNCHECKED;
    return;
  }
  const QGlob<IO> q{static_cast<const IO*>(a.q), a.ld, i, dof_of<Model>(C)};
  a.verdict[i] = V_FREE;
  if (Model::broad_flag(q, C)) idx[queue_q<Model>(q, count, qbuf, cap)] = int32_t(i);
}

struct VjpArgs {
  const DevProblem* P;
  int64_t n;
  const void* q;
  int64_t ld;
  const int8_t* status;
  const void* g;
  void* g_in;
  double cond_thr;
  unsigned int* defer_count;  // FP32 mode: configurations left to the FP64 tail kernel
  int32_t* defer_idx;
};

// The VJP kernels keep the upstream gradient g of a lane in LDS, in the precision of the solve (a
// [D][64] tile per wave after the waves' FP64 iterate tiles), instead of in registers across the Gram
// and the factorisation, and stream g_in = g - J^T y out of the J^T y walk joint by joint.
template <class S>
struct GLds {
  using LP = __attribute__((address_space(3))) S*;
  LP base;
  __device__ __forceinline__ S operator[](int j) const { return base[j * 64]; }
  __device__ __forceinline__ void set(int j, S v) const { base[j * 64] = v; }
};
// The calling lane's column of g: smem holds blockDim.x / 64 FP64 iterate tiles, then as many g tiles.
template <int D, class S>
__device__ __forceinline__ GLds<S> g_lds(double* smem) {
  const int w = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  S* base = reinterpret_cast<S*>(smem + (blockDim.x >> 6) * (D * 64)) + w * (D * 64) + l;
  return GLds<S>{(typename GLds<S>::LP)base};
}
// Sink of the J^T y walk: out[j] = acc stores g_in[j] = g[j] - acc (coordinates below dof).
template <class IO, class S>
struct VjpOut {
  IO* dst;  // g_in + i
  int64_t ld;
  GLds<S> g;
  int dof;
  struct Ref {
    const VjpOut* o;
    int j;
    __device__ __forceinline__ void operator=(S acc) const {
      if (j < o->dof) o->dst[int64_t(j) * o->ld] = IO(double(o->g[j]) - double(acc));
    }
  };
  __device__ __forceinline__ Ref operator[](int j) const { return Ref{this, j}; }
};

template <class Model, class IO, class S>
__device__ __forceinline__ void vjp_load(const VjpArgs& a, int dof, int64_t i, const QLds& q, const GLds<S>& g) {
  const IO* pq = static_cast<const IO*>(a.q) + i;
  const IO* pg = static_cast<const IO*>(a.g) + i;
  for (int c = 0; c < Model::D; ++c) {
    q.set(c, c < dof ? double(*pq) : 0.0);
    g.set(c, c < dof ? S(*pg) : S(0));
    const int64_t ld = after(a.ld, c);
    pq += ld;
    pg += ld;
  }
}

template <class IO>
__device__ __forceinline__ void vjp_fill(const VjpArgs& a, int dof, int64_t i, double v) {
  IO* p = static_cast<IO*>(a.g_in) + i;
  for (int c = 0; c < dof; ++c) p[int64_t(c) * a.ld] = IO(v);
}

// FP64 Gram, factorisation and projection for one lane: g_in = g - J^T (J J^T)^-1 J g (NaN where
// the FP64 factorisation fails).
template <class Model, class IO>
__device__ __forceinline__ void vjp64(const VjpArgs& a, int dof, int64_t i, const QLds& q, const GLds<double>& g,
                                      const Consts& C) {
  constexpr int M = Model::M;
  typename Model::template SD<double> sd;
  double F[M], G[M * (M + 1) / 2], v[M], invd[M], kappa;
  Model::template residual<double>(q, C, F, sd);
  Model::template gram<double, false>(q, C, sd, G, g, v);
  Model::template jv<double>(q, C, sd, g, v);
  double maxd = 0.0;
  for (int r = 0; r < M; ++r) maxd = fmax(maxd, G[pidx(r, r)]);
  if (cholesky<Model, double>(G, invd, kappa, kFloorF64 * maxd, drop_bits<Model>(sd))) {
    chol_solve<Model, double>(G, invd, v);
    Model::template jty<double>(q, C, sd, v, VjpOut<IO, double>{static_cast<IO*>(a.g_in) + i, a.ld, g, dof});
  } else {
    vjp_fill<IO>(a, dof, i, __builtin_nan(""));
  }
}

// g_in = g - J^T (J J^T)^-1 J g at the converged configuration (J recomputed; the forward
// pass stores nothing beyond q and status). g_in = 0 for configurations that did not converge.
// In FP32 mode a lane whose factorisation fails or whose condition estimate exceeds the
// threshold is queued for k_vjp_tail, which redoes it in FP64.
// Dynamic LDS: D * blockDim doubles (iterates) + D * blockDim S (gradients).
template <class Model, class IO, class S>
__global__ void __launch_bounds__(64) k_vjp(VjpArgs a) {
  constexpr int D = Model::D, M = Model::M;
  extern __shared__ double smem[];
  const Consts& C = consts_of(a.P);
  const QLds q = q_lds<D>(smem);
  const GLds<S> g = g_lds<D, S>(smem);
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int dof = dof_of<Model>(C);
  if (a.status[i] != ST_CONVERGED) {
    vjp_fill<IO>(a, dof, i, 0.0);
    return;
  }
  vjp_load<Model, IO, S>(a, dof, i, q, g);
  if constexpr (std::is_same<S, float>::value) {
    typename Model::template SD<float> sd;
    float F[M], G[M * (M + 1) / 2], v[M], invd[M], kappa;
    Model::template residual<float>(q, C, F, sd);
    Model::template gram<float, false>(q, C, sd, G, g, v);
    Model::template jv<float>(q, C, sd, g, v);
    if (cholesky<Model, float>(G, invd, kappa, kFloorF32, drop_bits<Model>(sd)) && double(kappa) <= a.cond_thr) {
      chol_solve<Model, float>(G, invd, v);
      Model::template jty<float>(q, C, sd, v, VjpOut<IO, float>{static_cast<IO*>(a.g_in) + i, a.ld, g, dof});
    } else {
      atomicAdd(a.P->fallback_counter, 1ull);
      a.defer_idx[atomicAdd(a.defer_count, 1u)] = int32_t(i);
    }
  } else {
    vjp64<Model, IO>(a, dof, i, q, g, C);
  }
}

// FP64 redo of the VJPs queued by k_vjp (grid-stride over the queue).
// Dynamic LDS: 2 * D * blockDim doubles (iterates, gradients).
template <class Model, class IO>
__global__ void __launch_bounds__(64) k_vjp_tail(VjpArgs a) {
  constexpr int D = Model::D;
  extern __shared__ double smem[];
  const Consts& C = consts_of(a.P);
  const int dof = dof_of<Model>(C);
  const QLds q = q_lds<D>(smem);
  const GLds<double> g = g_lds<D, double>(smem);
  const int64_t cnt = *a.defer_count;
  for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < cnt; s += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = a.defer_idx[s];
    vjp_load<Model, IO, double>(a, dof, i, q, g);
    vjp64<Model, IO>(a, dof, i, q, g, C);
  }
}

// ---------------------------------------------------------------- exact VJP off the manifold
// The derivative of the projection map itself (not only of the projection at its output), by
// reverse mode through the Newton steps the forward pass took: with q_{k+1} = q_k - alpha J^T y,
// y = G^-1 F, G = J J^T + lambda I, a cotangent w of q_{k+1} pulls back to
//   w_k = w - alpha (J^T z + H(y.F) a - H(z.F) delta),   z = G^-1 J w, a = w - J^T z, delta = J^T y,
// where H(c.F) v is the Hessian-vector product of the scalar c.F, the directional derivative of its
// gradient J^T c along v (here by central differences of the analytic gradient in FP64). The output
// cotangent is first projected on the tangent space at q_K, which is what one more Newton step at
// the converged point does to it (the converged map's derivative there).
struct VjpxArgs {
  const DevProblem* P;
  int64_t n;
  const void* q_in;   // the forward pass's (unprojected) inputs
  int64_t ld;
  const int8_t* status;
  const int8_t* iters;  // the forward pass's step counts
  const void* g;
  void* g_in;
  double alpha, lambda, h_rel;
};

// A per-lane FP32 column of a [D][64] LDS tile.
struct FLds {
  using LP = __attribute__((address_space(3))) float*;
  LP base;
  __device__ __forceinline__ float operator[](int j) const { return base[j * 64]; }
  __device__ __forceinline__ void set(int j, float v) const { base[j * 64] = v; }
};
// Sink of a J^T c walk that hands (j, value) to a callable.
template <class S, class Fn>
struct FnSink {
  Fn fn;
  struct Ref {
    const FnSink* o;
    int j;
    __device__ __forceinline__ void operator=(S acc) const { o->fn(j, acc); }
  };
  __device__ __forceinline__ Ref operator[](int j) const { return Ref{this, j}; }
};
template <class S, class Fn>
__device__ __forceinline__ FnSink<S, Fn> fn_sink(Fn fn) { return FnSink<S, Fn>{fn}; }
// The iterate moved along a unit direction: coordinate j is q_j + t u_j / |u|.
struct QShift {
  QLds q;
  FLds u;
  double t;  // step already divided by |u|
  __device__ __forceinline__ double at(int j) const { return q.at(j) + t * double(u[j]); }
  template <class U>
  __device__ __forceinline__ double at(int j, U dep) const { return q.at(j, dep) + t * double(u[j]); }
};

// FP64 Gram of J J^T + lambda I at q, factorised; false when it is not positive definite.
template <class Model>
__device__ __forceinline__ bool gram64(const QLds& q, const Consts& C, double lambda,
                                       typename Model::template SD<double>& sd, double* F, double* G, double* invd) {
  constexpr int M = Model::M;
  Model::template residual<double>(q, C, F, sd);
  Model::template gram<double, false>(q, C, sd, G, (const double*)nullptr, (double*)nullptr);
  double maxd = 0.0, kappa;
  for (int r = 0; r < M; ++r) {
    G[pidx(r, r)] += lambda;
    maxd = fmax(maxd, G[pidx(r, r)]);
  }
  return cholesky<Model, double>(G, invd, kappa, kFloorF64 * maxd, drop_bits<Model>(sd));
}

// k FP64 Newton steps from the input (replaying the forward pass's path); false on a failure.
template <class Model, class IO>
__device__ __forceinline__ bool replay(const VjpxArgs& a, int dof, int64_t i, int k, const QLds& q, const Consts& C) {
  constexpr int M = Model::M;
  const IO* p = static_cast<const IO*>(a.q_in) + i;
  for (int c = 0; c < Model::D; ++c) q.set(c, c < dof ? double(p[int64_t(c) * a.ld]) : 0.0);
  for (int s = 0; s < k; ++s) {
    typename Model::template SD<double> sd;
    double F[M], G[M * (M + 1) / 2], invd[M];
    if (!gram64<Model>(q, C, a.lambda, sd, F, G, invd)) return false;
    chol_solve<Model, double>(G, invd, F);
    const double al = a.alpha;
    // the walk has read coordinate j when it reports column j, so the update can go in place
    Model::template jty<double>(q, C, sd, F, fn_sink<double>([&](int j, double acc) { q.set(j, q.at(j) - al * acc); }));
  }
  return true;
}

// Accumulate coef * (gradient of c.F at q + t u/|u|) into w (the FP64 cotangent tile: the two
// evaluations of a central difference add nearly cancelling terms of size |u| |grad| / 2h).
// Rows that a lane may drop keep the base point's choice (base: the step data at q).
template <class Model>
__device__ __forceinline__ void grad_axpy(const QLds& q, const FLds& u, double t, const Consts& C, const double* c,
                                          double coef, const QLds& w, const typename Model::template SD<double>& base) {
  constexpr int M = Model::M;
  const QShift qs{q, u, t};
  typename Model::template SD<double> sd;
  double F[M];
  Model::template residual<double>(qs, C, F, sd);
  if constexpr (Model::DROPPABLE != 0) Model::freeze_rows(sd, base);
  Model::template jty<double>(qs, C, sd, c, fn_sink<double>([&](int j, double acc) { w.set(j, w.at(j) + coef * acc); }));
}

template <class Model, class IO>
__global__ void __launch_bounds__(64) k_vjp_exact(VjpxArgs a) {
  constexpr int D = Model::D, M = Model::M;
  extern __shared__ double smem[];
  const Consts& C = consts_of(a.P);
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int dof = dof_of<Model>(C);
  IO* out = static_cast<IO*>(a.g_in) + i;
  if (a.status[i] != ST_CONVERGED) {
    for (int c = 0; c < dof; ++c) out[int64_t(c) * a.ld] = IO(0);
    return;
  }
  // tiles: the FP64 iterate and cotangent w (waves' tiles in turn), then the FP32 direction v (a, then delta)
  const int nw = int(blockDim.x) >> 6, w0 = int(threadIdx.x) >> 6, l = int(threadIdx.x) & 63;
  const QLds q{(QLds::LP)(smem + w0 * (D * 64) + l)};
  const QLds w{(QLds::LP)(smem + (nw + w0) * (D * 64) + l)};
  float* fb = reinterpret_cast<float*>(smem + 2 * nw * (D * 64));
  const FLds v{(FLds::LP)(fb + w0 * (D * 64) + l)};
  const int K = a.iters[i];
  bool ok = replay<Model, IO>(a, dof, i, K, q, C);
  {
    const IO* pg = static_cast<const IO*>(a.g) + i;
    for (int c = 0; c < D; ++c) w.set(c, c < dof ? double(pg[int64_t(c) * a.ld]) : 0.0);
  }
  // w <- (I - J^+ J) w at q_K
  if (ok) {
    typename Model::template SD<double> sd;
    double F[M], G[M * (M + 1) / 2], invd[M], z[M];
    ok = gram64<Model>(q, C, 0.0, sd, F, G, invd);
    if (ok) {
      Model::template jv<double>(q, C, sd, w, z);
      chol_solve<Model, double>(G, invd, z);
      Model::template jty<double>(q, C, sd, z, fn_sink<double>([&](int j, double acc) { w.set(j, w.at(j) - acc); }));
    }
  }
  for (int k = K - 1; k >= 0 && ok; --k) {
    ok = replay<Model, IO>(a, dof, i, k, q, C);
    if (!ok) break;
    typename Model::template SD<double> sd;
    double F[M], G[M * (M + 1) / 2], invd[M], z[M];
    ok = gram64<Model>(q, C, a.lambda, sd, F, G, invd);
    if (!ok) break;
    chol_solve<Model, double>(G, invd, F);  // F <- y
    Model::template jv<double>(q, C, sd, w, z);
    chol_solve<Model, double>(G, invd, z);  // z = G^-1 J w
    const double al = a.alpha;
    // v <- a = w - J^T z, then w <- (1 - alpha) w + alpha a (= w - alpha J^T z)
    Model::template jty<double>(q, C, sd, z, fn_sink<double>([&](int j, double acc) {
      const double wj = w.at(j), aj = wj - acc;
      v.set(j, float(aj));
      w.set(j, (1.0 - al) * wj + al * aj);
    }));
    double qn = 1.0, vn = 0.0;
    for (int c = 0; c < D; ++c) {
      qn = fmax(qn, fabs(q.at(c)));
      vn += double(v[c]) * double(v[c]);
    }
    const double h = a.h_rel * qn;
    vn = sqrt(vn);
    // w -= alpha H(y.F) a: central difference of the gradient J^T y along a / |a|, times |a| / 2h
    if (vn > 0.0) {
      const double coef = al * vn / (2.0 * h);
      grad_axpy<Model>(q, v, h / vn, C, F, -coef, w, sd);
      grad_axpy<Model>(q, v, -h / vn, C, F, coef, w, sd);
    }
    // v <- delta = J^T y, then w += alpha H(z.F) delta
    Model::template jty<double>(q, C, sd, F, fn_sink<double>([&](int j, double acc) { v.set(j, float(acc)); }));
    double dn = 0.0;
    for (int c = 0; c < D; ++c) dn += double(v[c]) * double(v[c]);
    dn = sqrt(dn);
    if (dn > 0.0) {
      const double coef = al * dn / (2.0 * h);
      grad_axpy<Model>(q, v, h / dn, C, z, coef, w, sd);
      grad_axpy<Model>(q, v, -h / dn, C, z, -coef, w, sd);
    }
  }
  for (int c = 0; c < dof; ++c) out[int64_t(c) * a.ld] = ok ? IO(w.at(c)) : IO(__builtin_nan(""));
}

// Diagnostic: residual (FP64) and dense Jacobian (step precision S) as the projection
// kernels compute them.
template <class Model, class IO, class S>
__global__ void __launch_bounds__(256) k_eval_fj(const DevProblem* Pp, int64_t n, const void* qv, int64_t ld, void* Fo, void* Jo) {
  constexpr int D = Model::D, M = Model::M;
  const Consts& P = consts_of(Pp);
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int dof = P.dof, m = P.rows;
  const QGlob<IO> q{static_cast<const IO*>(qv), ld, i, dof};
  typename Model::template SD<double> sd64;
  double F[M];
  Model::template residual<double>(q, P, F, sd64);
  typename Model::template SD<S> sd;
  S Fs[M], J[M * D];
  Model::template residual<S>(q, P, Fs, sd);
  Model::template jacobian<S>(q, P, sd, J);
  for (int r = 0; r < M; ++r) {
    if (r >= m) continue;
    st_io<IO>(Fo, r * ld + i, F[r]);
    for (int c = 0; c < D; ++c)
      if (c < dof) st_io<IO>(Jo, (int64_t(r) * dof + c) * ld + i, double(J[r * D + c]));
  }
}

// Diagnostic: the condition estimate (max L_ii / min L_ii)^2 of J J^T + lambda I as the step
// computes it in precision S (+inf where the factorisation fails). The iterate is staged in LDS
// as in the projection kernels. Dynamic LDS: D * blockDim doubles.
template <class Model, class IO, class S>
__global__ void __launch_bounds__(64) k_eval_cond(const DevProblem* Pp, int64_t n, const void* qv, int64_t ld,
                                                  double lambda, void* kappa_out) {
  constexpr int D = Model::D, M = Model::M;
  extern __shared__ double smem[];
  const Consts& C = consts_of(Pp);
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int dof = dof_of<Model>(C);
  const QLds q = q_lds<D>(smem);
  const IO* p = static_cast<const IO*>(qv) + i;
  for (int c = 0; c < D; ++c) q.set(c, c < dof ? double(p[int64_t(c) * ld]) : 0.0);
  typename Model::template SD<S> sd;
  S F[M], G[M * (M + 1) / 2], invd[M], kappa;
  Model::template residual<S>(q, C, F, sd);
  Model::template gram<S, false>(q, C, sd, G, nullptr, nullptr);
  S maxd = S(0);
  for (int r = 0; r < M; ++r) {
    G[pidx(r, r)] += S(lambda);
    maxd = G[pidx(r, r)] > maxd ? G[pidx(r, r)] : maxd;
  }
  const S floor = std::is_same<S, float>::value ? S(kFloorF32) : S(kFloorF64);
  const bool ok = cholesky<Model, S>(G, invd, kappa, floor * maxd, drop_bits<Model>(sd));
  st_io<IO>(kappa_out, i, ok ? double(kappa) : __builtin_huge_val());
}

}  // namespace mc
