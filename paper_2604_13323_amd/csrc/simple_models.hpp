// Constraint models without a kinematic tree: the unit sphere F = q.q - 1
// (configuration = point robot) and linear constraints F = A q - b.
#pragma once

#include "common.hpp"

namespace mc {

// Point-robot sphere test against the grouped, clustered obstacles (group and cluster boxes,
// then the obstacles of overlapping clusters), or the exhaustive minimum signed distance.
template <bool MINSD>
__device__ __forceinline__ void point_check(const float* c, float r, const CollConsts& K, const float4* obs, bool& hit,
                                            float& minsd) {
  if constexpr (MINSD) {
    for (int o = 0; o < K.n_obs; ++o) {
      const float4 ob = obs[o];
      const float dx = c[0] - ob.x, dy = c[1] - ob.y, dz = c[2] - ob.z;
      const float d2 = dx * dx + dy * dy + dz * dz;
      const float rr = r + ob.w;
      hit = hit || (d2 < rr * rr);
      minsd = fminf(minsd, __fsqrt_rn(d2) - rr);
    }
  } else {
    for (int g = 0; g < K.n_sup; ++g) {
      if (!__any(!hit && box_dist2(c, K.sup_lo[g], K.sup_hi[g]) <= r * r)) continue;  // wave-uniform
      const int2 cr = K.sup_range[g];
      for (int k = cr.x; k < cr.y; ++k) {
        if (!hit && box_dist2(c, K.clus_lo[k], K.clus_hi[k]) <= r * r) {
          const int2 rg = K.clus_range[k];
          for (int o = rg.x; o < rg.y; ++o) {
            const float4 ob = obs[o];
            const float ex = c[0] - ob.x, ey = c[1] - ob.y, ez = c[2] - ob.z;
            const float r2 = r + ob.w;
            hit = hit || (ex * ex + ey * ey + ez * ez < r2 * r2);
          }
        }
      }
    }
  }
}

struct SphereModel {
  static constexpr int family = 0;
  static constexpr bool broad_in_residual = false;  // the exact check is cheap: run it at convergence
  static constexpr int D = 3, M = 1;
  static constexpr bool fixed_dof = false;  // the scene's d (at most D) is read at run time
  static constexpr int NBLK = 1;
  static constexpr uint32_t DROPPABLE = 0;  // no row is ever dropped
  static constexpr uint32_t ALL = ~uint32_t(0);
  static constexpr uint32_t block_rows_mask(int) { return ALL; }
  static constexpr bool lnz(int, int) { return true; }
  template <class S> struct SD { S dummy; };

  template <class S, uint32_t RM = ~uint32_t(0), class Q>
  static __device__ __forceinline__ double residual(const Q& q, const Consts&, S* F, SD<S>&) {
    const double a = q.at(0), b = q.at(1), c = q.at(2);
    const double f = a * a + b * b + c * c - 1.0;
    F[0] = S(f);
    return f * f;
  }
  // J = 2 q^T, so J J^T = 4 q.q and J g = 2 q.g
  template <class S, bool WITH_V, uint32_t RM = ~uint32_t(0), class Q, class GV = const S*>
  static __device__ __forceinline__ void gram(const Q& q, const Consts&, const SD<S>&, S* G, GV g, S* v) {
    const S a = S(q.at(0)), b = S(q.at(1)), c = S(q.at(2));
    G[0] = S(4) * (a * a + b * b + c * c);
    if constexpr (WITH_V) v[0] = S(2) * (a * g[0] + b * g[1] + c * g[2]);
  }
  template <class S, class Q, class GV>
  static __device__ __forceinline__ void jv(const Q& q, const Consts&, const SD<S>&, GV g, S* v) {
    v[0] = S(2) * (S(q.at(0)) * g[0] + S(q.at(1)) * g[1] + S(q.at(2)) * g[2]);
  }
  template <class S, uint32_t RM = ~uint32_t(0), class Q, class OUT>
  static __device__ __forceinline__ void jty(const Q& q, const Consts&, const SD<S>&, const S* y, OUT&& out) {
    for (int k = 0; k < 3; ++k) out[k] = S(2) * S(q.at(k)) * y[0];
  }
  template <class S, class Q>
  static __device__ __forceinline__ void jacobian(const Q& q, const Consts&, const SD<S>&, S* J) {
    for (int k = 0; k < 3; ++k) J[k] = S(2) * S(q.at(k));
  }
  template <class Q>
  static __device__ __forceinline__ bool broad_flag(const Q&, const Consts&) { return true; }
  // Point robot: every lane of the group runs the whole (cheap) test.
  template <int L, class Q>
  static __device__ __forceinline__ bool check_group(const Q& q, const Consts&, const CollConsts& K, const float4*,
                                                     const float4* obs, int part = 0, int = 1, float4* = nullptr) {
    if (part != 0) return false;  // a point robot's check is not split
    bool hit = false;
    float minsd;
    const float4 ps = K.point_sph;
    const float c[3] = {float(q.at(0)) + ps.x, float(q.at(1)) + ps.y, float(q.at(2)) + ps.z};
    point_check<false>(c, ps.w, K, obs, hit, minsd);
    return hit;
  }
  template <class Q>
  static __device__ __forceinline__ void min_signed_distance(const Q& q, const Consts&, const CollConsts& K,
                                                             const float4* obs, bool& hit, float& minsd) {
    hit = false;
    minsd = __builtin_huge_valf();
    const float4 ps = K.point_sph;
    const float c[3] = {float(q.at(0)) + ps.x, float(q.at(1)) + ps.y, float(q.at(2)) + ps.z};
    point_check<true>(c, ps.w, K, obs, hit, minsd);
  }
};

// F = A q - b with d <= LIN_D, m <= LIN_M. Arrays are padded to LIN_D / LIN_M: the padding
// columns of A are zero and the padding rows get an identity Gram block and a zero residual,
// so they contribute nothing to the step.
struct LinearModel {
  static constexpr int family = 1;
  static constexpr bool broad_in_residual = false;  // the exact check is cheap: run it at convergence
  static constexpr int D = LIN_D, M = LIN_M;
  static constexpr bool fixed_dof = false;  // the scene's d (at most D) is read at run time
  static constexpr int NBLK = 1;
  static constexpr uint32_t DROPPABLE = 0;  // no row is ever dropped
  static constexpr uint32_t ALL = ~uint32_t(0);
  static constexpr uint32_t block_rows_mask(int) { return ALL; }
  static constexpr bool lnz(int, int) { return true; }
  template <class S> struct SD { S dummy; };

  template <class S, uint32_t RM = ~uint32_t(0), class Q>
  static __device__ __forceinline__ double residual(const Q& q, const Consts& P, S* F, SD<S>&) {
    double qv[D], n2 = 0.0;
    for (int c = 0; c < D; ++c) qv[c] = q.at(c);
    for (int r = 0; r < M; ++r) {
      double acc = -P.d.b[r];
      for (int c = 0; c < D; ++c) acc += P.d.A[r][c] * qv[c];
      acc = r < P.lin_m ? acc : 0.0;
      F[r] = S(acc);
      n2 += acc * acc;
    }
    return n2;
  }
  template <class S, bool WITH_V, uint32_t RM = ~uint32_t(0), class Q, class GV = const S*>
  static __device__ __forceinline__ void gram(const Q&, const Consts& P, const SD<S>&, S* G, GV g, S* v) {
    const TP<S>& T = tp<S>(P);
    for (int i = 0; i < M; ++i) {
      for (int k = 0; k <= i; ++k) {
        S acc = S(0);
        for (int c = 0; c < D; ++c) acc += T.A[i][c] * T.A[k][c];
        G[pidx(i, k)] = (i >= P.lin_m) ? S(i == k ? 1 : 0) : acc;
      }
      if constexpr (WITH_V) {
        S acc = S(0);
        for (int c = 0; c < D; ++c) acc += T.A[i][c] * g[c];
        v[i] = i < P.lin_m ? acc : S(0);
      }
    }
  }
  template <class S, class Q, class GV>
  static __device__ __forceinline__ void jv(const Q&, const Consts& P, const SD<S>&, GV g, S* v) {
    const TP<S>& T = tp<S>(P);
    for (int i = 0; i < M; ++i) {
      S acc = S(0);
      for (int c = 0; c < D; ++c) acc += T.A[i][c] * g[c];
      v[i] = i < P.lin_m ? acc : S(0);
    }
  }
  template <class S, uint32_t RM = ~uint32_t(0), class Q, class OUT>
  static __device__ __forceinline__ void jty(const Q&, const Consts& P, const SD<S>&, const S* y, OUT&& out) {
    const TP<S>& T = tp<S>(P);
    for (int c = 0; c < D; ++c) {
      S acc = S(0);
      for (int r = 0; r < M; ++r) acc += T.A[r][c] * y[r];
      out[c] = acc;
    }
  }
  template <class S, class Q>
  static __device__ __forceinline__ void jacobian(const Q&, const Consts& P, const SD<S>&, S* J) {
    const TP<S>& T = tp<S>(P);
    for (int r = 0; r < M; ++r)
      for (int c = 0; c < D; ++c) J[r * D + c] = T.A[r][c];
  }
  template <int L, class Q>
  static __device__ __forceinline__ bool check_group(const Q&, const Consts&, const CollConsts&, const float4*,
                                                     const float4*, int = 0, int = 1, float4* = nullptr) {
    return false;
  }
  template <class Q>
  static __device__ __forceinline__ bool broad_flag(const Q&, const Consts&) { return false; }
  template <class Q>
  static __device__ __forceinline__ void min_signed_distance(const Q&, const Consts&, const CollConsts&, const float4*,
                                                             bool& hit, float& minsd) {
    hit = false;
    minsd = __builtin_huge_valf();
  }
};

}  // namespace mc
