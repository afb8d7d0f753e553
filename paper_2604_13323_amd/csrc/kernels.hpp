// Generic HIP kernels of the projection path, templated on the constraint model.
//
// Mapping: one configuration per lane; the lane's FP64 iterate lives in LDS (a column
// of a [D][blockDim] array, conflict-free), everything else in registers. The hot
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
  unsigned int* counter;  // persistent: queue head (reset to 0 before the launch)
  int64_t n_static;       // persistent: configurations [0, n_static) are taken by thread id
};

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
// In-place right-looking Cholesky of the packed lower triangle G (structural zeros of the
// factor skipped at compile time). Returns false on a non-positive or non-finite pivot, or a
// pivot below floor. invd receives 1 / L_ii; kappa the estimate (max L_ii / min L_ii)^2.
template <class Model, class S>
__device__ __forceinline__ bool cholesky(S* G, S* invd, S& kappa, S floor) {
  constexpr int M = Model::M;
  bool ok = true;
  S dmin = S(3.0e38), dmax = S(0);
  sfor<0, M>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const S d = G[pidx(k, k)];
    ok = ok && (d > floor) && finite_t(d);
    const S r = rsqrt_t(d);
    const S l = d * r;
    G[pidx(k, k)] = l;
    invd[k] = r;
    dmin = l < dmin ? l : dmin;
    dmax = l > dmax ? l : dmax;
    sfor<k + 1, M>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (Model::lnz(i, k)) G[pidx(i, k)] *= r;
    });
    sfor<k + 1, M>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (Model::lnz(i, k)) {
        sfor<k + 1, i + 1>([&](auto Jx) {
          constexpr int j = decltype(Jx)::value;
          if constexpr (Model::lnz(j, k)) G[pidx(i, j)] -= G[pidx(i, k)] * G[pidx(j, k)];
        });
      }
    });
  });
  const S ratio = dmax / dmin;
  kappa = ratio * ratio;
  return ok && finite_t(kappa);
}

// Solve L L^T y = b in place (b overwritten by y).
template <class Model, class S>
__device__ __forceinline__ void chol_solve(const S* L, const S* invd, S* y) {
  constexpr int M = Model::M;
  sfor<0, M>([&](auto I) {
    constexpr int i = decltype(I)::value;
    S acc = y[i];
    sfor<0, i>([&](auto K) {
      constexpr int k = decltype(K)::value;
      if constexpr (Model::lnz(i, k)) acc -= L[pidx(i, k)] * y[k];
    });
    y[i] = acc * invd[i];
  });
  sfor<0, M>([&](auto I) {
    constexpr int i = M - 1 - decltype(I)::value;
    S acc = y[i];
    sfor<i + 1, M>([&](auto K) {
      constexpr int k = decltype(K)::value;
      if constexpr (Model::lnz(k, i)) acc -= L[pidx(k, i)] * y[k];
    });
    y[i] = acc * invd[i];
  });
}

constexpr float kFloorF32 = 0.0f;
constexpr double kFloorF64 = 1e-24;  // pivot floor relative to the largest Gram diagonal entry

// One descent step in precision S: dq = J^T (J J^T + lambda I)^-1 rhs (rhs = F for Newton;
// overwritten). Returns false when the factorisation fails or its condition estimate
// exceeds cond_thr.
template <class Model, class S, class Q>
__device__ __forceinline__ bool descent_step(const Q& q, S* rhs, const typename Model::template SD<S>& sd,
                                             const DevProblem* Pp, double lambda, double cond_thr, S floor_rel, S* dq) {
  constexpr int M = Model::M;
  S G[M * (M + 1) / 2];
  Model::template gram<S, false>(q, cparams(Pp), sd, G, nullptr, nullptr);
  S maxd = S(0);
  sfor<0, M>([&](auto I) {
    constexpr int i = decltype(I)::value;
    G[pidx(i, i)] += S(lambda);
    maxd = G[pidx(i, i)] > maxd ? G[pidx(i, i)] : maxd;
  });
  S invd[M], kappa;
  if (!cholesky<Model, S>(G, invd, kappa, floor_rel * maxd)) return false;
  if (!(double(kappa) <= cond_thr)) return false;
  chol_solve<Model, S>(G, invd, rhs);
  Model::template jty<S>(q, cparams(Pp), sd, rhs, dq);
  return true;
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

// The whole step in FP64 for one lane (condition estimate above threshold or a failed FP32
// factorisation). Kept out of line so its register needs do not shape the FP32 path.
template <class Model>
__device__ __noinline__ int fp64_step(QLds q, const ProjArgs* ap) {
  const ProjArgs& a = *ap;
  typename Model::template SD<double> sd;
  double F[Model::M], dq[Model::D];
  Model::template residual<double>(q, cparams(a.P), F, sd);
  if (!descent_step<Model, double>(q, F, sd, a.P, a.lambda, 1e300, kFloorF64, dq)) return ST_SINGULAR;
  return apply_step<Model, double>(q, dq, a);
}

// One Newton iteration for one lane. Returns -1 after taking a step, else the final status.
template <class Model, class S>
__device__ __forceinline__ int newton_iteration(const QLds& q, int& k, const ProjArgs& a, double& resid) {
  constexpr int D = Model::D, M = Model::M;
  typename Model::template SD<S> sd;
  S F[M];
  const double n2 = Model::template residual<S>(q, cparams(a.P), F, sd);
  resid = sqrt(n2);
  if (!finite_t(n2)) return ST_NONFINITE;
  if (n2 < a.tol2) return ST_CONVERGED;
  if (k >= a.max_iter) return ST_MAX_ITER;
  int st;
  if constexpr (std::is_same<S, float>::value) {
    float dq[D];
    if (descent_step<Model, float>(q, F, sd, a.P, a.lambda, a.cond_thr, kFloorF32, dq)) {
      st = apply_step<Model, float>(q, dq, a);
    } else {
      atomicAdd(a.P->fallback_counter, 1ull);
#ifdef MC_EXPERIMENT_NO_FALLBACK
      st = ST_SINGULAR;
#else
      st = fp64_step<Model>(q, &a);
#endif
    }
  } else {
    double dq[D];
    if (descent_step<Model, double>(q, F, sd, a.P, a.lambda, 1e300, kFloorF64, dq))
      st = apply_step<Model, double>(q, dq, a);
    else
      st = ST_SINGULAR;
  }
  if (st < 0) ++k;
  return st;
}

template <class Model, class IO>
__device__ __forceinline__ void load_q(const ProjArgs& a, int64_t i, const QLds& q) {
  const int dof = a.P->dof;
  for (int c = 0; c < Model::D; ++c) q.set(c, c < dof ? ld_io<IO>(a.q_in, c * a.ld_in + a.base + i) : 0.0);
}

template <class Model, class IO>
__device__ __forceinline__ void store_result(const ProjArgs& a, int64_t i, const QLds& q, int st, int k, double resid) {
  const int dof = a.P->dof;
  for (int c = 0; c < Model::D; ++c)
    if (c < dof) st_io<IO>(a.q_out, c * a.ld_out + a.base + i, q.at(c));
  a.status[a.base + i] = int8_t(st);
  a.iters[a.base + i] = int8_t(k);
  st_io<IO>(a.resid, a.base + i, resid);
}

// Persistent projection kernel: a grid of resident waves pulls configurations from a device
// work queue (atomic counter), one per lane, and refills a lane when its configuration ends.
// Dynamic LDS: D * blockDim doubles.
template <class Model, class IO, class S>
__global__ void __launch_bounds__(256) k_project_persistent(ProjArgs a) {
  extern __shared__ double smem[];
  const QLds q{smem + threadIdx.x, int(blockDim.x)};
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n_static) i = a.n;  // not part of the static share
  int k = 0;
  if (i < a.n) load_q<Model, IO>(a, i, q);
  for (;;) {
    const bool active = i < a.n;
    if (!__any(active)) break;
    if (active) {
      double resid;
      const int st = newton_iteration<Model, S>(q, k, a, resid);
      if (st >= 0) {
        store_result<Model, IO>(a, i, q, st, k, resid);
        i = a.n_static + int64_t(atomicAdd(a.counter, 1u));
        k = 0;
        if (i < a.n) load_q<Model, IO>(a, i, q);
      }
    }
  }
}

// Plain kernel: one launch per geodesic, one configuration per lane, projection and
// collision check in the same kernel, no work queue.
template <class Model, class IO, class S>
__global__ void __launch_bounds__(64) k_project_plain(ProjArgs a) {
  extern __shared__ double smem[];
  const QLds q{smem + threadIdx.x, int(blockDim.x)};
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  load_q<Model, IO>(a, i, q);
  int k = 0, st;
  double resid;
  for (;;) {
    st = newton_iteration<Model, S>(q, k, a, resid);
    if (st >= 0) break;
  }
  store_result<Model, IO>(a, i, q, st, k, resid);
  if (a.verdict) {
    uint8_t v = V_UNCHECKED;
    if (a.check && st == ST_CONVERGED) {
      bool hit;
      float msd;
      Model::template check<false>(q, cparams(a.P), hit, msd);
      v = hit ? V_HIT : V_FREE;
    }
    a.verdict[a.base + i] = v;
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

template <class Model, class IO, bool MINSD>
__global__ void __launch_bounds__(256) k_check(CheckArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  if (a.status && a.status[i] != ST_CONVERGED) {
    a.verdict[i] = V_UNCHECKED;
    return;
  }
  const QGlob<IO> q{static_cast<const IO*>(a.q), a.ld, i, a.P->dof};
  bool hit;
  float msd;
  Model::template check<MINSD>(q, cparams(a.P), hit, msd);
  a.verdict[i] = hit ? V_HIT : V_FREE;
  if constexpr (MINSD) st_io<IO>(a.minsd, i, double(msd));
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
};

// FP64 Gram, factorisation and projection for one lane (condition estimate above threshold).
template <class Model>
__device__ __noinline__ void vjp64(QLds q, const VjpArgs* ap, const double* gd, double* out) {
  constexpr int D = Model::D, M = Model::M;
  const VjpArgs& a = *ap;
  typename Model::template SD<double> sd;
  double F[M], G[M * (M + 1) / 2], v[M], invd[M], kappa, jy[D];
  Model::template residual<double>(q, cparams(a.P), F, sd);
  Model::template gram<double, true>(q, cparams(a.P), sd, G, gd, v);
  double maxd = 0.0;
  for (int r = 0; r < M; ++r) maxd = fmax(maxd, G[pidx(r, r)]);
  if (cholesky<Model, double>(G, invd, kappa, kFloorF64 * maxd)) {
    chol_solve<Model, double>(G, invd, v);
    Model::template jty<double>(q, cparams(a.P), sd, v, jy);
    for (int j = 0; j < D; ++j) out[j] = gd[j] - jy[j];
  } else {
    for (int j = 0; j < D; ++j) out[j] = __builtin_nan("");
  }
}

// g_in = g - J^T (J J^T)^-1 J g at the converged configuration (J recomputed; the forward
// pass stores nothing beyond q and status).
template <class Model, class IO, class S>
__global__ void __launch_bounds__(256) k_vjp(VjpArgs a) {
  constexpr int D = Model::D, M = Model::M;
  extern __shared__ double smem[];
  const QLds q{smem + threadIdx.x, int(blockDim.x)};
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int dof = a.P->dof;
  if (a.status[i] != ST_CONVERGED) {
    for (int c = 0; c < D; ++c)
      if (c < dof) st_io<IO>(a.g_in, c * a.ld + i, 0.0);
    return;
  }
  double gd[D];
  for (int c = 0; c < D; ++c) {
    q.set(c, c < dof ? ld_io<IO>(a.q, c * a.ld + i) : 0.0);
    gd[c] = c < dof ? ld_io<IO>(a.g, c * a.ld + i) : 0.0;
  }
  double out[D];
  bool done = false;
  if constexpr (std::is_same<S, float>::value) {
    typename Model::template SD<float> sd;
    float F[M], gs[D], G[M * (M + 1) / 2], v[M], invd[M], kappa;
    Model::template residual<float>(q, cparams(a.P), F, sd);
    for (int j = 0; j < D; ++j) gs[j] = float(gd[j]);
    Model::template gram<float, true>(q, cparams(a.P), sd, G, gs, v);
    if (cholesky<Model, float>(G, invd, kappa, kFloorF32) && double(kappa) <= a.cond_thr) {
      chol_solve<Model, float>(G, invd, v);
      float jy[D];
      Model::template jty<float>(q, cparams(a.P), sd, v, jy);
      for (int j = 0; j < D; ++j) out[j] = gd[j] - double(jy[j]);
      done = true;
    } else {
      atomicAdd(a.P->fallback_counter, 1ull);
    }
  }
  if (!done) vjp64<Model>(q, &a, gd, out);
  for (int c = 0; c < D; ++c)
    if (c < dof) st_io<IO>(a.g_in, c * a.ld + i, out[c]);
}

// Diagnostic: residual (FP64) and dense Jacobian (step precision S) as the projection
// kernels compute them.
template <class Model, class IO, class S>
__global__ void __launch_bounds__(256) k_eval_fj(const DevProblem* Pp, int64_t n, const void* qv, int64_t ld, void* Fo, void* Jo) {
  constexpr int D = Model::D, M = Model::M;
  const DevProblem& P = cparams(Pp);
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

}  // namespace mc
