// Kinematic-tree constraint models with compile-time topology.
//
// The paper traces each robot's kinematics into straight-line SIMD code with no
// branches or loops (Sec. IV-A, tracing compiler). Here the same effect comes
// from C++ templates: a robot's joint tree, joint types and
// axes, end-effector frames and constraint blocks are constexpr data, and every
// loop over joints, rows and Gram entries is unrolled at compile time with the
// structural zeros of the Jacobian, the Gram matrix and its Cholesky factor
// removed. Numeric parameters (origins, masses, targets) stay runtime data read
// with wave-uniform (scalar) loads.
//
// Conventions: joint j has parent p(j) (-1 = world), fixed origin O_j and axis
// a_j of its own frame; the link frame is T_j = T_p(j) O_j Q_j(q_j). Joints are
// in depth-first preorder, so the subtree of j is the index range [j, end_j).
// A revolute joint's world axis is z_j = R_j e_{a_j} and its origin o_j = p_j.
//
// Residual blocks (rows stacked in block order):
//   POSE  (Eq. 1)  T_err = T_ref^-1 T_f, rows [t; log(R)^v] selected by a mask.
//   REL   (Eq. 2)  T_err = T_ref^-1 (T_a^-1 T_b), rows [t; log(R)^v].
//   AXIS           (R_f e_z)_x, (R_f e_z)_y  (frame z-axis parallel to world z).
//   COM   (Digit constraint figure, equality form) sum_l m_l c_l / M |_xy - target.
//   HULL  (Digit constraint figure) that CoM xy minus its nearest point of a convex polygon, zero
//         inside; in an edge region written in the edge's frame, [n.d, 0].
//   DIST  (Digit constraint figure, closed linkage) ||p_b - p_a|| - L between two frame origins.
//   A POSE block flagged BF_BOUNDED has finite bounds: a row is its component's excess over the
//   interval [lo, hi].
// Rows that vanish on a region (a bounded component inside its interval, polygon rows inside the
// polygon, the second polygon row of an edge region) are dropped per lane: zero residual, zero
// Jacobian row, and a unit Cholesky pivot, so the step is the minimum-norm step of the rows left.
//
// Analytic Jacobian columns (for a revolute joint j; prismatic in brackets):
//   POSE  [W (z_j x (p_f - o_j)); A z_j]    [W z_j; 0],   W = R_ref^T, A = J_l^-1(w) W
//   REL   s_j [W (z_j x (p_b - o_j)); A z_j] with W = (R_a R_ref)^T, s_j = +1 when j moves
//         only frame b, -1 when it moves only frame a, 0 when it moves both
//   AXIS  (z_j x u)_xy with u = R_f e_z         [0]
//   COM   (z_j x (S_j - M_j o_j))_xy / M        [(M_j / M) z_j,xy]
//         S_j = sum of m_l c_l over the subtree of j, M_j its mass.
//   HULL  H c with c the COM column and H the lane's 2 x 2 row map (edge frame, identity, or 0;
//         its lower-left entry is always 0)
//   DIST  s_j u.(z_j x (p_e - o_j)), p_e the moving end   [s_j u.z_j],  u = (p_b - p_a) / |p_b - p_a|
#pragma once

#include "common.hpp"

namespace mc {

// ------------------------------------------------------------------ topologies
struct TopoPlanar2 {
  static constexpr int family = 2;
  static constexpr int NJ = 2, NF = 1, NB = 1, M = 2;
  static constexpr int parent[NJ] = {-1, 0};
  static constexpr int jtype[NJ] = {REV, REV};
  static constexpr int axis[NJ] = {2, 2};
  static constexpr bool origin_rot = false, frame_rot = false;
  static constexpr int frame_link[NF] = {1};
  static constexpr int btype[NB] = {B_POSE};
  static constexpr int bfa[NB] = {0};
  static constexpr int bfb[NB] = {-1};
  static constexpr int bmask[NB] = {0x3};
  static constexpr int bflags[NB] = {0};
  static constexpr bool has_com = false;
  static constexpr bool massless(int) { return true; }
  static constexpr bool may_have_spheres(int) { return true; }
};

struct TopoArm7Axis {
  static constexpr int family = 3;
  static constexpr int NJ = 7, NF = 1, NB = 1, M = 2;
  static constexpr int parent[NJ] = {-1, 0, 1, 2, 3, 4, 5};
  static constexpr int jtype[NJ] = {REV, REV, REV, REV, REV, REV, REV};
  static constexpr int axis[NJ] = {2, 2, 2, 2, 2, 2, 2};
  static constexpr bool origin_rot = true, frame_rot = true;
  static constexpr int frame_link[NF] = {6};
  static constexpr int btype[NB] = {B_AXIS};
  static constexpr int bfa[NB] = {0};
  static constexpr int bfb[NB] = {-1};
  static constexpr int bmask[NB] = {0};
  static constexpr int bflags[NB] = {0};
  static constexpr bool has_com = false;
  static constexpr bool massless(int) { return true; }
  static constexpr bool may_have_spheres(int) { return true; }
};

struct TopoDual14Rel {
  static constexpr int family = 4;
  static constexpr int persist_waves = 2;  // the FP32 stacked projection fits 256 registers per lane
  static constexpr int NJ = 14, NF = 2, NB = 1, M = 6;
  static constexpr int parent[NJ] = {-1, 0, 1, 2, 3, 4, 5, -1, 7, 8, 9, 10, 11, 12};
  static constexpr int jtype[NJ] = {REV, REV, REV, REV, REV, REV, REV, REV, REV, REV, REV, REV, REV, REV};
  static constexpr int axis[NJ] = {2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
  static constexpr bool origin_rot = true, frame_rot = true;
  static constexpr int frame_link[NF] = {6, 13};
  static constexpr int btype[NB] = {B_REL};
  static constexpr int bfa[NB] = {0};
  static constexpr int bfb[NB] = {1};
  static constexpr int bmask[NB] = {0x3F};
  static constexpr int bflags[NB] = {0};
  static constexpr bool has_com = false;
  static constexpr bool massless(int) { return true; }
  static constexpr bool may_have_spheres(int) { return true; }
};

// 6-DoF floating base (Px Py Pz Rz Ry Rx -> pelvis = link 5), legs 2 x 6, torso 2,
// arms 2 x 7, head 2.
struct TopoHumanoid36 {
  static constexpr int family = 5;
  static constexpr int NJ = 36, NF = 4, NB = 4, M = 20;
  static constexpr int parent[NJ] = {-1, 0, 1, 2, 3, 4,
                                     5, 6, 7, 8, 9, 10,
                                     5, 12, 13, 14, 15, 16,
                                     5, 18,
                                     19, 20, 21, 22, 23, 24, 25,
                                     19, 27, 28, 29, 30, 31, 32,
                                     19, 34};
  static constexpr int jtype[NJ] = {PRI, PRI, PRI, REV, REV, REV,
                                    REV, REV, REV, REV, REV, REV,
                                    REV, REV, REV, REV, REV, REV,
                                    REV, REV,
                                    REV, REV, REV, REV, REV, REV, REV,
                                    REV, REV, REV, REV, REV, REV, REV,
                                    REV, REV};
  static constexpr int axis[NJ] = {0, 1, 2, 2, 1, 0,
                                   2, 0, 1, 1, 1, 0,
                                   2, 0, 1, 1, 1, 0,
                                   2, 1,
                                   1, 0, 2, 1, 2, 1, 0,
                                   1, 0, 2, 1, 2, 1, 0,
                                   2, 1};
  static constexpr bool origin_rot = false, frame_rot = false;
  static constexpr int frame_link[NF] = {11, 17, 26, 33};   // left sole, right sole, left palm, right palm
  static constexpr int btype[NB] = {B_POSE, B_POSE, B_REL, B_COM};
  static constexpr int bfa[NB] = {0, 1, 2, -1};
  static constexpr int bfb[NB] = {-1, -1, 3, -1};
  static constexpr int bmask[NB] = {0x3F, 0x3F, 0x3F, 0};
  static constexpr int bflags[NB] = {0, 0, 0, 0};
  static constexpr bool has_com = true;
  static constexpr bool massless(int j) { return j < 5; }     // the base's intermediate links
  static constexpr bool may_have_spheres(int j) { return j >= 5; }
};

// The humanoid tree with the Digit constraint set: feet poses, hands relative pose, CoM within the
// support polygon, and one closed-linkage rod per leg (hip-roll link to shin).
struct TopoDigit36 {
  static constexpr int family = 6;
  static constexpr int NJ = 36, NF = 8, NB = 6, M = 22;
  static constexpr int parent[NJ] = {-1, 0, 1, 2, 3, 4,
                                     5, 6, 7, 8, 9, 10,
                                     5, 12, 13, 14, 15, 16,
                                     5, 18,
                                     19, 20, 21, 22, 23, 24, 25,
                                     19, 27, 28, 29, 30, 31, 32,
                                     19, 34};
  static constexpr int jtype[NJ] = {PRI, PRI, PRI, REV, REV, REV,
                                    REV, REV, REV, REV, REV, REV,
                                    REV, REV, REV, REV, REV, REV,
                                    REV, REV,
                                    REV, REV, REV, REV, REV, REV, REV,
                                    REV, REV, REV, REV, REV, REV, REV,
                                    REV, REV};
  static constexpr int axis[NJ] = {0, 1, 2, 2, 1, 0,
                                   2, 0, 1, 1, 1, 0,
                                   2, 0, 1, 1, 1, 0,
                                   2, 1,
                                   1, 0, 2, 1, 2, 1, 0,
                                   1, 0, 2, 1, 2, 1, 0,
                                   2, 1};
  static constexpr bool origin_rot = false, frame_rot = false;
  // left sole, right sole, left palm, right palm, rod ends: left hip, left shin, right hip, right shin
  static constexpr int frame_link[NF] = {11, 17, 26, 33, 7, 9, 13, 15};
  static constexpr int btype[NB] = {B_POSE, B_POSE, B_REL, B_HULL, B_DIST, B_DIST};
  static constexpr int bfa[NB] = {0, 1, 2, -1, 4, 6};
  static constexpr int bfb[NB] = {-1, -1, 3, -1, 5, 7};
  static constexpr int bmask[NB] = {0x3F, 0x3F, 0x3F, 0, 0, 0};
  static constexpr int bflags[NB] = {0, 0, 0, 0, 0, 0};
  static constexpr bool has_com = true;
  static constexpr bool massless(int j) { return j < 5; }
  static constexpr bool may_have_spheres(int j) { return j >= 5; }
};

// The 7-DoF arm with one TSR pose block of finite bounds on its end-effector frame (all six
// components; a free component has infinite bounds).
struct TopoArm7Tsr {
  static constexpr int family = 7;
  static constexpr int NJ = 7, NF = 1, NB = 1, M = 6;
  static constexpr int parent[NJ] = {-1, 0, 1, 2, 3, 4, 5};
  static constexpr int jtype[NJ] = {REV, REV, REV, REV, REV, REV, REV};
  static constexpr int axis[NJ] = {2, 2, 2, 2, 2, 2, 2};
  static constexpr bool origin_rot = true, frame_rot = true;
  static constexpr int frame_link[NF] = {6};
  static constexpr int btype[NB] = {B_POSE};
  static constexpr int bfa[NB] = {0};
  static constexpr int bfb[NB] = {-1};
  static constexpr int bmask[NB] = {0x3F};
  static constexpr int bflags[NB] = {BF_BOUNDED};
  static constexpr bool has_com = false;
  static constexpr bool massless(int) { return true; }
  static constexpr bool may_have_spheres(int) { return true; }
};

// ------------------------------------------------------------------ structure
template <class Topo>
struct KInfo {
  static constexpr int NJ = Topo::NJ, NB = Topo::NB, M = Topo::M;
  static constexpr bool anc(int j, int l) {
    for (int k = l; k >= 0; k = Topo::parent[k])
      if (k == j) return true;
    return false;
  }
  static constexpr int popc6(int x) {
    int c = 0;
    for (int i = 0; i < 6; ++i) c += (x >> i) & 1;
    return c;
  }
  static constexpr int brows(int b) {
    return (Topo::btype[b] == B_POSE || Topo::btype[b] == B_REL) ? popc6(Topo::bmask[b])
                                                                   : (Topo::btype[b] == B_DIST ? 1 : 2);
  }
  static constexpr int brow0(int b) {
    int r = 0;
    for (int k = 0; k < b; ++k) r += brows(k);
    return r;
  }
  static constexpr uint32_t brmask(int b) { return ((uint32_t(1) << brows(b)) - 1u) << brow0(b); }
  static constexpr int flink(int f) { return Topo::frame_link[f]; }
  // 0: block b does not depend on joint j; +-1: it does (sign for REL).
  static constexpr int dep(int b, int j) {
    const int t = Topo::btype[b];
    if (t == B_POSE) return anc(j, flink(Topo::bfa[b])) ? 1 : 0;
    if (t == B_AXIS) return (anc(j, flink(Topo::bfa[b])) && Topo::jtype[j] == REV) ? 1 : 0;
    if (t == B_REL || t == B_DIST) {
      const bool a = anc(j, flink(Topo::bfa[b])), bb = anc(j, flink(Topo::bfb[b]));
      return a == bb ? 0 : (bb ? 1 : -1);
    }
    if (t == B_COM || t == B_HULL) return 1;
    return 0;
  }
  static constexpr int row_block(int r) {
    for (int b = 0; b < NB; ++b)
      if (r < brow0(b) + brows(b)) return b;
    return -1;
  }
  // component (0..5 of [t; w] for pose blocks, 0..1 otherwise) of row r
  static constexpr int row_comp(int r) {
    const int b = row_block(r);
    const int k = r - brow0(b);
    if (Topo::btype[b] == B_POSE || Topo::btype[b] == B_REL) {
      int seen = 0;
      for (int c = 0; c < 6; ++c)
        if ((Topo::bmask[b] >> c) & 1) {
          if (seen == k) return c;
          ++seen;
        }
      return -1;
    }
    return k;
  }
  // row r is structurally nonzero in column j (tabulated once: the pattern computations below
  // query it many times)
  static constexpr bool rdep_eval(int r, int j) {
    const int b = row_block(r);
    if (dep(b, j) == 0) return false;
    const int t = Topo::btype[b];
    if ((t == B_POSE || t == B_REL) && row_comp(r) >= 3 && Topo::jtype[j] == PRI) return false;
    return true;
  }
  struct RD { bool v[MAXM][MAXJ]; };
  static constexpr RD rd_table() {
    RD t{};
    for (int r = 0; r < M; ++r)
      for (int j = 0; j < NJ; ++j) t.v[r][j] = rdep_eval(r, j);
    return t;
  }
  static constexpr RD RDT = rd_table();
  static constexpr bool rdep(int r, int j) { return RDT.v[r][j]; }
  static constexpr bool gnz(int r1, int r2) {
    for (int j = 0; j < NJ; ++j)
      if (rdep(r1, j) && rdep(r2, j)) return true;
    return false;
  }
  struct Pat { bool nz[MAXM][MAXM]; };
  static constexpr Pat lpattern() {
    Pat P{};
    for (int i = 0; i < M; ++i)
      for (int k = 0; k <= i; ++k) P.nz[i][k] = gnz(i, k);
    for (int k = 0; k < M; ++k)
      for (int i = k + 1; i < M; ++i)
        for (int j = k + 1; j <= i; ++j)
          if (P.nz[i][k] && P.nz[j][k]) P.nz[i][j] = true;
    return P;
  }
  static constexpr Pat LP = lpattern();
  static constexpr int sub_end(int j) {
    int e = j + 1;
    while (e < NJ && anc(j, e)) ++e;
    return e;
  }
  static constexpr bool end_needed(int e) {
    for (int j = 0; j < NJ; ++j)
      if (sub_end(j) == e) return true;
    return false;
  }
  static constexpr int complete_link(int b) {
    const int t = Topo::btype[b];
    if (t == B_POSE || t == B_AXIS) return flink(Topo::bfa[b]);
    if (t == B_REL || t == B_DIST)
      return flink(Topo::bfa[b]) > flink(Topo::bfb[b]) ? flink(Topo::bfa[b]) : flink(Topo::bfb[b]);
    return NJ - 1;
  }
  // rows that may be dropped per lane (bounded pose components, polygon rows)
  static constexpr bool droppable(int b) {
    return Topo::btype[b] == B_HULL || (Topo::btype[b] == B_POSE && (Topo::bflags[b] & BF_BOUNDED));
  }
  static constexpr uint32_t drop_rows() {
    uint32_t m = 0;
    for (int b = 0; b < NB; ++b)
      if (droppable(b)) m |= brmask(b);
    return m;
  }
};


// ------------------------------------------------------------------ model
// Kinematic constants are read with scalar loads (uniform values cost scalar registers, not
// vector registers), each joint's ordered after the walk reaches it.
template <class T, class U>
__device__ __forceinline__ const T& after_cp(const T& r, U dep) {
  return after_const(r, dep);
}

template <class Topo>
struct Kin {
  using KI = KInfo<Topo>;
  static constexpr int NJ = Topo::NJ, NB = Topo::NB, NF = Topo::NF, M = Topo::M, D = Topo::NJ;
  static constexpr bool fixed_dof = true;  // a scene of this family has exactly D coordinates
  static constexpr int family = Topo::family;
  static constexpr bool broad_in_residual = true;  // broad_flag() tests the link bounds against the obstacle box
  static constexpr int NBLK = NB;                  // constraint blocks (the cyclic mode steps them in order)
  static constexpr int persist_waves = PersistWaves<Topo>::value;
  static constexpr uint32_t ALL = ~uint32_t(0);
  static constexpr uint32_t block_rows_mask(int b) { return KI::brmask(b); }
  static constexpr uint32_t DROPPABLE = KI::drop_rows();  // rows a lane may drop (see the header)
  template <uint32_t RM>
  static constexpr bool sel(int b) { return (KI::brmask(b) & RM) != 0; }
  static constexpr bool in_rows(uint32_t rm, int r) { return (rm >> r) & 1u; }
  static constexpr bool lnz(int i, int k) { return KI::LP.nz[i][k]; }

  // Per-iteration data from the residual pass used by the Jacobian passes.
  template <class S>
  struct SD {
    S pend[NB][3];    // end point of pose / relative-pose blocks
    S W[NB][9];       // REL: (R_a R_ref)^T
    S A[NB][9];       // J_l^-1(w) W
    S u[NB][3];       // AXIS: frame z axis; DIST: unit vector from end a to end b
    S pa[NB][3];      // DIST: end a (pend holds end b)
    S H[NB][3];       // HULL: the lane's 2 x 2 row map [h0 h1; 0 h2]
    S Qe[NJ + 1][3];  // prefix sums of m_l c_l at the subtree ends
    uint32_t drop = 0;  // rows dropped in this lane (bits of DROPPABLE)
  };

  // Take the base point's choice of rows (dropped rows, polygon row map) into sd: the rows are then
  // the smooth piece that is active at the base point, which the central differences of the exact
  // VJP must differentiate even where a shifted point lies across a region boundary.
  template <class S>
  static __device__ __forceinline__ void freeze_rows(SD<S>& sd, const SD<S>& base) {
    sd.drop = base.drop;
    sfor<0, NB>([&](auto BI) {
      constexpr int b = decltype(BI)::value;
      if constexpr (Topo::btype[b] == B_HULL)
        for (int k = 0; k < 3; ++k) sd.H[b][k] = base.H[b][k];
    });
  }

  // Joint coordinate in the pass precision. FP32 passes take revolute angles reduced to
  // [-pi, pi] in FP64 first, so large angles keep full FP32 accuracy in sine and cosine.
  template <class T, int type>
  static __device__ __forceinline__ T joint_value(double x) {
    if constexpr (std::is_same<T, float>::value && type == REV) {
      const double k = __builtin_rint(x * 0.15915494309189535);  // 1 / (2 pi)
      x = __builtin_fma(-k, 6.283185307179586, x);
      x = __builtin_fma(-k, 2.4492935982947064e-16, x);
    }
    return T(x);
  }

  // What the walk needs at joint j, read with scalar loads one joint ahead of its use.
  template <class T>
  struct JP {
    T q;       // joint coordinate
    T p[3];    // origin translation
    T R[9];    // origin rotation (when the topology has rotated origins)
    T m;       // link mass
    T mc[3];   // mass * local CoM
  };

  template <class T, int j, class Q, class U>
  static __device__ __forceinline__ JP<T> load_joint(const Q& q, const TP<T>& P0, U dep) {
    JP<T> r;
    r.q = joint_value<T, Topo::jtype[j]>(q.at(j, dep));
    const TP<T>& P = after_cp(P0, dep);
    for (int k = 0; k < 3; ++k) r.p[k] = P.jp[j][k];
    if constexpr (Topo::origin_rot)
      for (int k = 0; k < 9; ++k) r.R[k] = P.jR[j][k];
    if constexpr (Topo::has_com && !Topo::massless(j)) {
      r.m = P.mass[j];
      for (int k = 0; k < 3; ++k) r.mc[k] = P.mcom[j][k];
    }
    return r;
  }

  // Forward kinematics, streaming each link frame to visit(ic<j>, frame, joint data) in joint
  // order. Joint j+1's data is read while joint j is computed; with ORDERED, joint j+1's read
  // is ordered after joint j-1's frame, so the walk keeps one joint of data in flight (register
  // budget of the projection passes); without, the compiler may issue every read up front (the
  // collision kernels, which have registers to spare and little arithmetic to hide latency).
  template <class T, bool ORDERED = true, class Q, class V>
  static __device__ __forceinline__ void fk(const Q& q, const TP<T>& P, V&& visit) {
    Rig<T> L[NJ];
    JP<T> cur = load_joint<T, 0>(q, P, 0);
    sfor<0, NJ>([&](auto J) {
      constexpr int j = decltype(J)::value;
      constexpr int par = Topo::parent[j];
      constexpr int ax = Topo::axis[j];
      JP<T> nxt;  // the next joint's data, requested one joint ahead
      if constexpr (j + 1 < NJ) {
        if constexpr (!ORDERED) nxt = load_joint<T, j + 1>(q, P, 0);
        else if constexpr (j > 0) nxt = load_joint<T, j + 1>(q, P, L[j - 1].p[2]);
        else nxt = load_joint<T, j + 1>(q, P, cur.q);
      }
      Rig<T>& X = L[j];
      if constexpr (par < 0) {
        if constexpr (Topo::origin_rot) {
          for (int k = 0; k < 9; ++k) X.R[k] = cur.R[k];
        } else {
          for (int k = 0; k < 9; ++k) X.R[k] = (k % 4 == 0) ? T(1) : T(0);
        }
        for (int k = 0; k < 3; ++k) X.p[k] = cur.p[k];
      } else {
        const Rig<T>& B = L[par];
        if constexpr (Topo::origin_rot) {
          matmul3(B.R, cur.R, X.R);
        } else {
          for (int k = 0; k < 9; ++k) X.R[k] = B.R[k];
        }
        T t[3];
        matvec3(B.R, cur.p, t);
        for (int k = 0; k < 3; ++k) X.p[k] = B.p[k] + t[k];
      }
      if constexpr (Topo::jtype[j] == PRI) {
        for (int r = 0; r < 3; ++r) X.p[r] += X.R[3 * r + ax] * cur.q;
      } else {
        T s, c;
        sincos_t(cur.q, &s, &c);
        constexpr int i = (ax + 1) % 3, k = (ax + 2) % 3;
        for (int r = 0; r < 3; ++r) {
          const T a = X.R[3 * r + i], b = X.R[3 * r + k];
          X.R[3 * r + i] = a * c + b * s;
          X.R[3 * r + k] = b * c - a * s;
        }
      }
      visit(J, X, cur);
      if constexpr (j + 1 < NJ) cur = nxt;
    });
  }

  template <class T>
  static __device__ __forceinline__ void frame_pose(const Rig<T>& X, const TP<T>& P0, int f, Rig<T>& out) {
    const TP<T>& P = after_cp(P0, X.p[2]);
    if constexpr (Topo::frame_rot) {
      matmul3(X.R, P.fR[f], out.R);
    } else {
      for (int k = 0; k < 9; ++k) out.R[k] = X.R[k];
    }
    T t[3];
    matvec3(X.R, P.fp[f], t);
    for (int k = 0; k < 3; ++k) out.p[k] = X.p[k] + t[k];
  }

  // rows of a pose error (t, log R) selected by the block mask
  template <int b, class S>
  static __device__ __forceinline__ void put_pose_rows(const double* t, const double* w, S* F, double& n2) {
    constexpr int r0 = KI::brow0(b);
    sfor<0, KI::brows(b)>([&](auto K) {
      constexpr int c = KI::row_comp(r0 + decltype(K)::value);
      const double v = c < 3 ? t[c] : w[c - 3];
      F[r0 + decltype(K)::value] = to_step<S>(v);
      n2 += v * v;
    });
  }

  // rows of a pose error with finite bounds: each component's excess over [lo, hi], dropped inside
  template <int b, class S>
  static __device__ __forceinline__ void put_bounded_rows(const double* t, const double* w, const TP<double>& Pd,
                                                          S* F, double& n2, uint32_t& drop) {
    constexpr int r0 = KI::brow0(b);
    sfor<0, KI::brows(b)>([&](auto K) {
      constexpr int r = r0 + decltype(K)::value;
      constexpr int c = KI::row_comp(r);
      const double v = c < 3 ? t[c] : w[c - 3];
      const double lo = Pd.blo[b][c], hi = Pd.bhi[b][c];
      const double e = v > hi ? v - hi : (v < lo ? v - lo : 0.0);
      const bool in = !(v > hi) && !(v < lo);
      drop = in ? (drop | (1u << r)) : (drop & ~(1u << r));
      F[r] = to_step<S>(e);
      n2 += e * e;
    });
  }

  template <class S, int b>
  static __device__ __forceinline__ void block_rows(const Rig<double>* Fr, const Consts& P0, S* F, double& n2, SD<S>& sd) {
    constexpr int t = Topo::btype[b];
    constexpr int r0 = KI::brow0(b);
    // the block's constants are read only once its frames exist
    constexpr int flast = (t == B_REL || t == B_DIST) ? Topo::bfb[b] : Topo::bfa[b];
    const Consts& P = after_cp(P0, Fr[flast < 0 ? 0 : flast].p[2]);
    if constexpr (t == B_POSE) {
      constexpr int fa = Topo::bfa[b];
      const double* Rt = P.d.refRt[b];
      double dp[3] = {Fr[fa].p[0] - P.d.refp[b][0], Fr[fa].p[1] - P.d.refp[b][1], Fr[fa].p[2] - P.d.refp[b][2]};
      double tt[3], Re[9], w[3], Jl[9], A[9];
      matvec3(Rt, dp, tt);
      matmul3(Rt, Fr[fa].R, Re);
      so3_log_jlinv(Re, w, Jl);
      if constexpr ((Topo::bflags[b] & BF_BOUNDED) != 0) put_bounded_rows<b>(tt, w, P.d, F, n2, sd.drop);
      else put_pose_rows<b>(tt, w, F, n2);
      matmul3(Jl, Rt, A);
      for (int k = 0; k < 3; ++k) sd.pend[b][k] = to_step<S>(Fr[fa].p[k]);
      for (int k = 0; k < 9; ++k) sd.A[b][k] = to_step<S>(A[k]);
    } else if constexpr (t == B_REL) {
      constexpr int fa = Topo::bfa[b], fb = Topo::bfb[b];
      const double* Rt = P.d.refRt[b];
      double W[9];  // W = R_ref^T R_a^T
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
          W[3 * i + k] = Rt[3 * i] * Fr[fa].R[3 * k] + Rt[3 * i + 1] * Fr[fa].R[3 * k + 1] + Rt[3 * i + 2] * Fr[fa].R[3 * k + 2];
      double dp[3] = {Fr[fb].p[0] - Fr[fa].p[0], Fr[fb].p[1] - Fr[fa].p[1], Fr[fb].p[2] - Fr[fa].p[2]};
      double tt[3], pr[3], Re[9], w[3], Jl[9], A[9];
      matvec3(W, dp, tt);
      matvec3(Rt, P.d.refp[b], pr);
      for (int k = 0; k < 3; ++k) tt[k] -= pr[k];
      matmul3(W, Fr[fb].R, Re);
      so3_log_jlinv(Re, w, Jl);
      put_pose_rows<b>(tt, w, F, n2);
      matmul3(Jl, W, A);
      for (int k = 0; k < 3; ++k) sd.pend[b][k] = to_step<S>(Fr[fb].p[k]);
      for (int k = 0; k < 9; ++k) sd.W[b][k] = to_step<S>(W[k]);
      for (int k = 0; k < 9; ++k) sd.A[b][k] = to_step<S>(A[k]);
    } else if constexpr (t == B_DIST) {
      constexpr int fa = Topo::bfa[b], fb = Topo::bfb[b];
      const double dv[3] = {Fr[fb].p[0] - Fr[fa].p[0], Fr[fb].p[1] - Fr[fa].p[1], Fr[fb].p[2] - Fr[fa].p[2]};
      const double len = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      const double e = len - P.d.target[b][0];
      F[r0] = to_step<S>(e);
      n2 += e * e;
      const double il = 1.0 / len;
      for (int k = 0; k < 3; ++k) {
        sd.u[b][k] = to_step<S>(dv[k] * il);
        sd.pend[b][k] = to_step<S>(Fr[fb].p[k]);
        sd.pa[b][k] = to_step<S>(Fr[fa].p[k]);
      }
    } else if constexpr (t == B_AXIS) {
      constexpr int fa = Topo::bfa[b];
      F[r0] = to_step<S>(Fr[fa].R[2]);
      F[r0 + 1] = to_step<S>(Fr[fa].R[5]);
      n2 += Fr[fa].R[2] * Fr[fa].R[2] + Fr[fa].R[5] * Fr[fa].R[5];
      sd.u[b][0] = to_step<S>(Fr[fa].R[2]);
      sd.u[b][1] = to_step<S>(Fr[fa].R[5]);
      sd.u[b][2] = to_step<S>(Fr[fa].R[8]);
    }
  }

  // Polygon rows of the CoM point (x, y): the nearest point of the polygon's boundary, edge by edge
  // (projection onto each segment, clamped to its ends). Inside (left of every edge): both rows
  // dropped. Nearest point inside an edge: rows [n.(x - c), 0] in the edge's frame, the second
  // dropped, row map H = [n; 0]. Nearest point a vertex v: rows x - v, H = I.
  template <class S, int b>
  // Each edge's constants are read after the previous edge's distance (scalar loads hoisted ahead
  // of the kinematic walk would hold registers through it).
  static __device__ __forceinline__ void hull_rows(double x, double y, const Consts& P0, S* F, double& n2, SD<S>& sd) {
    constexpr int r0 = KI::brow0(b);
    const Consts& P = after_cp(P0, y);
    const int nv = P.hull_nv;
    bool inside = true, on_edge = false;
    double best = 1e300, bx = 0.0, by = 0.0, bnx = 0.0, bny = 0.0;
    for (int i = 0; i < MAXHV; ++i) {
      if (i < nv) {
        const TP<double>& Pd = after_cp(P.d, best);
        const double* e = Pd.hull_e[i];
        const double* nn = Pd.hull_n[i];
        const double dx = x - e[0], dy = y - e[1];
        inside = inside && (e[2] * dy - e[3] * dx >= 0.0);
        const double t = (dx * e[2] + dy * e[3]) * nn[2];
        const double tc = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        const double cx = e[0] + tc * e[2], cy = e[1] + tc * e[3];
        const double d2 = (x - cx) * (x - cx) + (y - cy) * (y - cy);
        if (d2 < best) {
          best = d2;
          bx = cx;
          by = cy;
          on_edge = t > 0.0 && t < 1.0;
          bnx = nn[0];
          bny = nn[1];
        }
      }
    }
    // branch-free: inside, both rows dropped; edge region, [n.(x - c), 0] with the second dropped;
    // vertex region, x - v
    const bool vtx = !inside && !on_edge;
    const double dx = x - bx, dy = y - by;
    const double f0 = inside ? 0.0 : (on_edge ? bnx * dx + bny * dy : dx);
    const double f1 = vtx ? dy : 0.0;
    const double h0 = inside ? 0.0 : (on_edge ? bnx : 1.0);
    const double h1 = on_edge ? bny : 0.0;
    const double h3 = vtx ? 1.0 : 0.0;
    const uint32_t dm = inside ? 3u : (on_edge ? 2u : 0u);
    F[r0] = to_step<S>(f0);
    F[r0 + 1] = to_step<S>(f1);
    n2 += f0 * f0 + f1 * f1;
    sd.H[b][0] = to_step<S>(h0);
    sd.H[b][1] = to_step<S>(h1);
    sd.H[b][2] = to_step<S>(h3);
    sd.drop = (sd.drop & ~(3u << r0)) | (dm << r0);
  }

  // Residual pass in FP64: returns ||F(q)||^2 (FP64); F in the step precision S and the
  // step data for the Jacobian passes. RM selects the rows (blocks) to evaluate; the other
  // entries of F and sd are left untouched.
  template <class S, uint32_t RM = ALL, class Q>
  static __device__ __forceinline__ double residual(const Q& q, const Consts& P, S* F, SD<S>& sd) {
    Rig<double> Fr[NF];
    double cm[3] = {0.0, 0.0, 0.0};
    double n2 = 0.0;
    fk<double>(q, P.d, [&](auto J, const Rig<double>& X, const JP<double>& jp) {
      constexpr int j = decltype(J)::value;
      sfor<0, NF>([&](auto FI) {
        constexpr int f = decltype(FI)::value;
        if constexpr (Topo::frame_link[f] == j) frame_pose<double>(X, P.d, f, Fr[f]);
      });
      if constexpr (Topo::has_com) {
        if constexpr (!Topo::massless(j)) {
          double t[3];
          matvec3(X.R, jp.mc, t);
          // accumulated here, at its joint: the link's mass constants are then dead at once
          // instead of being kept (spilled) until the CoM rows at the end of the walk
          for (int k = 0; k < 3; ++k) cm[k] = opaque(cm[k] + t[k] + jp.m * X.p[k]);
        }
        if constexpr (KI::end_needed(j + 1)) {
          for (int k = 0; k < 3; ++k) sd.Qe[j + 1][k] = to_step<S>(cm[k]);
        }
      }
      sfor<0, NB>([&](auto BI) {
        constexpr int b = decltype(BI)::value;
        if constexpr (KI::complete_link(b) == j && sel<RM>(b)) block_rows<S, b>(Fr, P, F, n2, sd);
      });
    });
    sfor<0, NB>([&](auto BI) {
      constexpr int b = decltype(BI)::value;
      if constexpr (Topo::btype[b] == B_COM && sel<RM>(b)) {
        constexpr int r0 = KI::brow0(b);
        const TP<double>& Pd = after_cp(P.d, cm[1]);
        const double e0 = cm[0] * Pd.inv_total_mass - Pd.target[b][0];
        const double e1 = cm[1] * Pd.inv_total_mass - Pd.target[b][1];
        F[r0] = to_step<S>(e0);
        F[r0 + 1] = to_step<S>(e1);
        n2 += e0 * e0 + e1 * e1;
      } else if constexpr (Topo::btype[b] == B_HULL && sel<RM>(b)) {
        const TP<double>& Pd = after_cp(P.d, cm[1]);
        hull_rows<S, b>(cm[0] * Pd.inv_total_mass, cm[1] * Pd.inv_total_mass, P, F, n2, sd);
      }
    });
    return n2;
  }

  // Structurally nonzero entries of Jacobian column j (other rows untouched). Qr is the running
  // prefix sum of m_l c_l over the links before j and is advanced past link j.
  template <class S, int j, uint32_t RM = ALL>
  static __device__ __forceinline__ void column(const Rig<S>& X, const JP<S>& jp, const TP<S>& T, const SD<S>& sd,
                                                S* Qr, S* col) {
    constexpr int ax = Topo::axis[j];
    constexpr bool rev = Topo::jtype[j] == REV;
    const S z[3] = {X.R[ax], X.R[3 + ax], X.R[6 + ax]};
    const S* o = X.p;
    sfor<0, NB>([&](auto BI) {
      constexpr int b = decltype(BI)::value;
      constexpr int sg = sel<RM>(b) ? KI::dep(b, j) : 0;
      constexpr int t = Topo::btype[b];
      constexpr int r0 = KI::brow0(b);
      if constexpr (sg != 0 && (t == B_POSE || t == B_REL)) {
        S tv[3];
        if constexpr (rev) {
          const S r[3] = {sd.pend[b][0] - o[0], sd.pend[b][1] - o[1], sd.pend[b][2] - o[2]};
          cross3(z, r, tv);
        } else {
          tv[0] = z[0]; tv[1] = z[1]; tv[2] = z[2];
        }
        S lin[3], ang[3] = {S(0), S(0), S(0)};
        if constexpr (t == B_POSE) matvec3(T.refRt[b], tv, lin); else matvec3(sd.W[b], tv, lin);
        if constexpr (rev) matvec3(sd.A[b], z, ang);
        sfor<0, KI::brows(b)>([&](auto K) {
          constexpr int r = r0 + decltype(K)::value;
          constexpr int c = KI::row_comp(r);
          if constexpr (KI::rdep(r, j)) {
            const S v = c < 3 ? lin[c] : ang[c - 3];
            if constexpr (((DROPPABLE >> r) & 1u) != 0) col[r] = ((sd.drop >> r) & 1u) ? S(0) : (sg > 0 ? v : -v);
            else col[r] = sg > 0 ? v : -v;
          }
        });
      } else if constexpr (sg != 0 && t == B_DIST) {
        S v;
        if constexpr (rev) {
          const S* pe = sg > 0 ? sd.pend[b] : sd.pa[b];
          const S r[3] = {pe[0] - o[0], pe[1] - o[1], pe[2] - o[2]};
          S tv[3];
          cross3(z, r, tv);
          v = sd.u[b][0] * tv[0] + sd.u[b][1] * tv[1] + sd.u[b][2] * tv[2];
        } else {
          v = sd.u[b][0] * z[0] + sd.u[b][1] * z[1] + sd.u[b][2] * z[2];
        }
        col[r0] = sg > 0 ? v : -v;
      } else if constexpr (sg != 0 && t == B_AXIS) {
        col[r0] = z[1] * sd.u[b][2] - z[2] * sd.u[b][1];
        col[r0 + 1] = z[2] * sd.u[b][0] - z[0] * sd.u[b][2];
      } else if constexpr (sg != 0 && (t == B_COM || t == B_HULL)) {
        constexpr int e = KI::sub_end(j);
        const S iM = T.inv_total_mass;
        S c0, c1;
        if constexpr (rev) {
          const S Mj = T.submass[j];
          S Sp[3];
          for (int k = 0; k < 3; ++k) Sp[k] = sd.Qe[e][k] - Qr[k] - Mj * o[k];
          c0 = (z[1] * Sp[2] - z[2] * Sp[1]) * iM;
          c1 = (z[2] * Sp[0] - z[0] * Sp[2]) * iM;
        } else {
          const S f = T.submass[j] * iM;
          c0 = z[0] * f;
          c1 = z[1] * f;
        }
        if constexpr (t == B_COM) {
          col[r0] = c0;
          col[r0 + 1] = c1;
        } else {
          col[r0] = sd.H[b][0] * c0 + sd.H[b][1] * c1;
          col[r0 + 1] = sd.H[b][2] * c1;
        }
      }
    });
    if constexpr (Topo::has_com && !Topo::massless(j)) {
      S t[3];
      matvec3(X.R, jp.mc, t);
      for (int k = 0; k < 3; ++k) Qr[k] += t[k] + jp.m * X.p[k];
    }
  }

  // Gram pass: G += J_j J_j^T over all columns (packed lower triangle), optionally v = J g.
  template <class S, bool WITH_V, uint32_t RM = ALL, class Q, class GV = const S*>
  static __device__ __forceinline__ void gram(const Q& q, const Consts& P, const SD<S>& sd, S* G, GV g, S* v) {
    const TP<S>& T = tp<S>(P);
    sfor<0, M>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (in_rows(RM, i)) {
        sfor<0, i + 1>([&](auto K) {
          constexpr int k = decltype(K)::value;
          if constexpr (lnz(i, k) && in_rows(RM, k)) G[pidx(i, k)] = S(0);
        });
        if constexpr (WITH_V) v[i] = S(0);
      }
    });
    S Qr[3] = {S(0), S(0), S(0)};
    fk<S>(q, T, [&](auto J, const Rig<S>& X, const JP<S>& jp) {
      constexpr int j = decltype(J)::value;
      S col[M];
      column<S, j, RM>(X, jp, T, sd, Qr, col);
      sfor<0, M>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (KI::rdep(i, j) && in_rows(RM, i)) {
          sfor<0, i + 1>([&](auto K) {
            constexpr int k = decltype(K)::value;
            if constexpr (KI::rdep(k, j) && in_rows(RM, k)) G[pidx(i, k)] += col[i] * col[k];
          });
          if constexpr (WITH_V) v[i] += col[i] * g[j];
        }
      });
    });
  }

  // v = J g pass (its own walk: accumulating v inside the Gram walk keeps g and v live next to the
  // Gram and spills).
  template <class S, class Q, class GV>
  static __device__ __forceinline__ void jv(const Q& q, const Consts& P, const SD<S>& sd, GV g, S* v) {
    const TP<S>& T = tp<S>(P);
    for (int i = 0; i < M; ++i) v[i] = S(0);
    S Qr[3] = {S(0), S(0), S(0)};
    fk<S>(q, T, [&](auto J, const Rig<S>& X, const JP<S>& jp) {
      constexpr int j = decltype(J)::value;
      S col[M];
      column<S, j>(X, jp, T, sd, Qr, col);
      const S gj = g[j];
      sfor<0, M>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (KI::rdep(i, j)) v[i] += col[i] * gj;
      });
    });
  }

  // J^T y pass: out[j] = (J^T y)_j, assigned in joint order (out: an array, or a sink whose
  // operator[] returns an assignable proxy, so results can be streamed out of the walk).
  template <class S, uint32_t RM = ALL, class Q, class OUT>
  static __device__ __forceinline__ void jty(const Q& q, const Consts& P, const SD<S>& sd, const S* y, OUT&& out) {
    const TP<S>& T = tp<S>(P);
    S Qr[3] = {S(0), S(0), S(0)};
    fk<S>(q, T, [&](auto J, const Rig<S>& X, const JP<S>& jp) {
      constexpr int j = decltype(J)::value;
      S col[M];
      column<S, j, RM>(X, jp, T, sd, Qr, col);
      S acc = S(0);
      sfor<0, M>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (KI::rdep(i, j) && in_rows(RM, i)) acc += col[i] * y[i];
      });
      out[j] = acc;
    });
  }

  // Dense Jacobian (diagnostic): J[r * D + c].
  template <class S, class Q>
  static __device__ __forceinline__ void jacobian(const Q& q, const Consts& P, const SD<S>& sd, S* Jd) {
    const TP<S>& T = tp<S>(P);
    S Qr[3] = {S(0), S(0), S(0)};
    for (int k = 0; k < M * D; ++k) Jd[k] = S(0);
    fk<S>(q, T, [&](auto J, const Rig<S>& X, const JP<S>& jp) {
      constexpr int j = decltype(J)::value;
      S col[M];
      column<S, j>(X, jp, T, sd, Qr, col);
      sfor<0, M>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (KI::rdep(i, j)) Jd[i * D + j] = col[i];
      });
    });
  }

  // ---------------------------------------------------------------- collision check
  // Links that carry spheres in this topology (compile-time slots; a runtime sphere range may
  // still be empty).
  static constexpr int NGEO = [] {
    int n = 0;
    for (int l = 0; l < NJ; ++l) n += Topo::may_have_spheres(l) ? 1 : 0;
    return n;
  }();

  // Rank of link l among the links that may carry spheres.
  static constexpr int geo_rank(int l) {
    int n = 0;
    for (int k = 0; k < l; ++k) n += Topo::may_have_spheres(k) ? 1 : 0;
    return n;
  }

  // Exact sphere test of one link's spheres (world frame X) against obstacles [o0, o1).
  template <bool MINSD>
  static __device__ __forceinline__ void narrow(const Rig<float>& X, const CollConsts& K, const float4* obs, int l,
                                                int o0, int o1, bool& hit, float& minsd) {
    const int s0 = K.sph_begin[l], s1 = K.sph_begin[l + 1];
    for (int s = s0; s < s1; ++s) {
      const float4 sp = K.sph[s];
      const float lc[3] = {sp.x, sp.y, sp.z};
      float c[3];
      matvec3(X.R, lc, c);
      for (int k = 0; k < 3; ++k) c[k] += X.p[k];
      for (int o = o0; o < o1; ++o) {
        const float4 ob = obs[o];
        const float dx = c[0] - ob.x, dy = c[1] - ob.y, dz = c[2] - ob.z;
        const float d2 = dx * dx + dy * dy + dz * dz;
        const float rr = sp.w + ob.w;
        hit = hit || (d2 < rr * rr);
        if constexpr (MINSD) minsd = fminf(minsd, __fsqrt_rn(d2) - rr);
      }
    }
  }

  // Collision check of one configuration (robot spheres vs obstacle spheres, strict overlap) by
  // a group of L consecutive lanes that all hold the same configuration (L = 1, 2, 4, ..., 64).
  // Lane t of the group owns clusters t, t + L, ... (the boxes of its first slots are loaded once,
  // before the walk, and kept in registers). The walk streams each link frame; for a link with spheres every
  // lane tests the link's bounding sphere against its clusters' boxes, a ballot gives the group
  // the clusters the link overlaps, and for each of those the L lanes share the exact tests of the
  // link's spheres (sph) against the cluster's obstacles (obs). sph and obs may point to LDS
  // copies. Returns the verdict (the same in all L lanes).
  // With parts > 1 the group handles only the links of rank part, part + parts, ... (the other
  // parts of the configuration's check run in other groups).
  template <int L, class Q>
  static __device__ __forceinline__ bool check_group(const Q& q, const Consts& P, const CollConsts& K,
                                                     const float4* sph, const float4* obs, int part = 0,
                                                     int parts = 1, float4* slots = nullptr) {
    static_assert(L >= 1 && L <= 64 && (L & (L - 1)) == 0, "L must be a power of two <= 64");
    constexpr int PB = (MAXC + L - 1) / L < 8 ? (MAXC + L - 1) / L : 8;  // boxes kept in registers
    const int lane = int(__lane_id());
    const int t = lane & (L - 1);
    const int shift = lane & ~(L - 1);
    const uint64_t gmask = L == 64 ? ~uint64_t(0) : ((uint64_t(1) << L) - 1);
    const int ncl = K.n_clus;
    const int nb = (ncl + L - 1) / L;  // cluster slots per lane
    float4 blo[PB], bhi[PB];
    // one wave per configuration with at most 64 clusters: each lane also keeps its cluster's
    // obstacle range, so the pair loop below fetches it with a cross-lane read instead of a
    // dependent scalar load per overlapping cluster
    const bool ranges_in_lanes = L == 64 && ncl <= 64;
    int2 my_rg = make_int2(0, 0);
    if (ranges_in_lanes && t < ncl) my_rg = K.clus_range[t];
    sfor<0, PB>([&](auto BI) {
      constexpr int bi = decltype(BI)::value;
      const int c = bi * L + t;
      blo[bi] = c < ncl ? K.clus_lo[c] : make_float4(1e30f, 1e30f, 1e30f, 0.f);  // empty box
      bhi[bi] = c < ncl ? K.clus_hi[c] : make_float4(-1e30f, -1e30f, -1e30f, 0.f);
    });
    bool hit = false;
    fk<float, false>(q, P.f, [&](auto J, const Rig<float>& X, const JP<float>&) {
      constexpr int l = decltype(J)::value;
      if constexpr (Topo::may_have_spheres(l)) {
        const float4 bs = K.link_bs[l];
        // a group that already has its verdict skips the remaining links
        const bool done = ((uint64_t(__ballot(hit)) >> shift) & gmask) != 0;
        const bool mine = parts == 1 || geo_rank(l) % parts == part;
        if (bs.w >= 0.f && !done && mine) {
          const float lc[3] = {bs.x, bs.y, bs.z};
          float cb[3];
          matvec3(X.R, lc, cb);
          for (int k = 0; k < 3; ++k) cb[k] += X.p[k];
          const float r2 = bs.w * bs.w;
          const int s0 = K.sph_begin[l], ns = K.sph_begin[l + 1] - s0;
          // exact tests of the link against cluster cc (obstacles rg), in all L lanes of the group
          auto pairs = [&](int cc, int2 rg) {
            const int no = rg.y - rg.x;
            if constexpr (L <= 16) {
              // each sphere's centre once, tested against the cluster's box first (the box bounds
              // the obstacle spheres with a margin far above FP32 rounding, so a sphere farther
              // than its radius from it overlaps none of them); the group's lanes split the
              // obstacles of the spheres that pass
              const float4 clo = K.clus_lo[cc], chi = K.clus_hi[cc];
              for (int si = 0; si < ns; ++si) {
                const float4 sp = sph[s0 + si];
                const float lp[3] = {sp.x, sp.y, sp.z};
                float w[3];
                matvec3(X.R, lp, w);
                const float c[3] = {w[0] + X.p[0], w[1] + X.p[1], w[2] + X.p[2]};
                if (box_dist2(c, clo, chi) > sp.w * sp.w) continue;
                for (int oi = t; oi < no; oi += L) {
                  const float4 ob = obs[rg.x + oi];
                  const float dx = c[0] - ob.x, dy = c[1] - ob.y, dz = c[2] - ob.z;
                  const float rr = sp.w + ob.w;
                  hit = hit || (dx * dx + dy * dy + dz * dz < rr * rr);
                }
              }
            } else if (slots != nullptr && ns <= L) {
              // a wave per configuration: lane t transforms sphere t and tests it against the
              // cluster's box; the candidates' centres go to the wave's LDS slots in rank order
              // and the lanes split the (candidate, obstacle) pairs
              const float4 clo = K.clus_lo[cc], chi = K.clus_hi[cc];
              bool cand = false;
              float4 cs = make_float4(0.f, 0.f, 0.f, 0.f);
              if (t < ns) {
                const float4 sp = sph[s0 + t];
                const float lp[3] = {sp.x, sp.y, sp.z};
                float w[3];
                matvec3(X.R, lp, w);
                const float c[3] = {w[0] + X.p[0], w[1] + X.p[1], w[2] + X.p[2]};
                cand = box_dist2(c, clo, chi) <= sp.w * sp.w;
                cs = make_float4(c[0], c[1], c[2], sp.w);
              }
              const uint64_t cm = (uint64_t(__ballot(cand)) >> shift) & gmask;
              if (cand) slots[__popcll(cm & ((uint64_t(1) << t) - 1))] = cs;
              const int np = __popcll(cm) * no;
              for (int pi = t; pi < np; pi += L) {
                const int k = pi / no, oi = pi - k * no;
                const float4 c = slots[k];
                const float4 ob = obs[rg.x + oi];
                const float dx = c.x - ob.x, dy = c.y - ob.y, dz = c.z - ob.z;
                const float rr = c.w + ob.w;
                hit = hit || (dx * dx + dy * dy + dz * dz < rr * rr);
              }
            } else {
              // a wave per configuration: the link's sphere-obstacle pairs flattened over the lanes
              const int np = ns * no;
              for (int pi = t; pi < np; pi += L) {
                const int si = pi / no, oi = pi - si * no;
                const float4 sp = sph[s0 + si];
                const float4 ob = obs[rg.x + oi];
                const float lp[3] = {sp.x, sp.y, sp.z};
                float w[3];
                matvec3(X.R, lp, w);
                const float dx = w[0] + X.p[0] - ob.x, dy = w[1] + X.p[1] - ob.y, dz = w[2] + X.p[2] - ob.z;
                const float rr = sp.w + ob.w;
                hit = hit || (dx * dx + dy * dy + dz * dz < rr * rr);
              }
            }
          };
          // the clusters of slot b that some lane of the group found overlapping
          auto process = [&](int b, bool ov) {
            uint64_t m = (uint64_t(__ballot(ov)) >> shift) & gmask;
            while (m) {  // the same list in all L lanes
              const int cc = b * L + __builtin_ctzll(m);
              m &= m - 1;
              int2 rg;
              if (ranges_in_lanes) {
                rg.x = __shfl(my_rg.x, cc);
                rg.y = __shfl(my_rg.y, cc);
              } else {
                rg = K.clus_range[cc];
              }
              pairs(cc, rg);
            }
          };
          if constexpr (L == 1) {
            // one lane per configuration: the link's bound against the boxes of the cluster groups
            // first, then against the clusters of the groups it reaches (a group's box contains its
            // clusters' boxes, in FP32 too, so no overlapping cluster is skipped)
            for (int g = 0; g < K.n_sup; ++g) {
              if (box_dist2(cb, K.sup_lo[g], K.sup_hi[g]) > r2) continue;
              const int2 gr = K.sup_range[g];
              for (int c = gr.x; c < gr.y; ++c)
                if (box_dist2(cb, K.clus_lo[c], K.clus_hi[c]) <= r2) pairs(c, K.clus_range[c]);
            }
            return;
          }
          uint32_t own = 0;  // bit b: this lane's cluster of slot b overlaps the link's bound
          sfor<0, PB>([&](auto BI) {
            constexpr int bi = decltype(BI)::value;
            own |= uint32_t(box_dist2(cb, blo[bi], bhi[bi]) <= r2) << bi;
          });
          const int nbp = nb < PB ? nb : PB;
          for (int b = 0; b < nbp; ++b) process(b, (own >> b) & 1u);
          for (int b = PB; b < nb; ++b) {  // clusters beyond the register-resident ones
            const int c = b * L + t;
            process(b, c < ncl && box_dist2(cb, K.clus_lo[c], K.clus_hi[c]) <= r2);
          }
        }
      }
    });
    return ((uint64_t(__ballot(hit)) >> shift) & gmask) != 0;
  }

  // Broad-phase flag of one configuration: does the bounding sphere of some link reach into the
  // box around all obstacles? (FP32 walk; the link bounds and the box are inflated by a margin
  // that covers FP32 rounding, so a clear flag proves the configuration collision-free.)
  template <class Q>
  static __device__ __forceinline__ bool broad_flag(const Q& q, const Consts& P) {
    int nr = 0;
    fk<float, false>(q, P.f, [&](auto J, const Rig<float>& X, const JP<float>&) {
      constexpr int l = decltype(J)::value;
      if constexpr (Topo::may_have_spheres(l)) {
        const TP<float>& T = P.f;
        const float4 blo = make_float4(T.obs_lo[0], T.obs_lo[1], T.obs_lo[2], 0.f);
        const float4 bhi = make_float4(T.obs_hi[0], T.obs_hi[1], T.obs_hi[2], 0.f);
        const float* bs = T.lbs[l];
        float c[3];
        for (int k = 0; k < 3; ++k) c[k] = X.p[k] + X.R[3 * k] * bs[0] + X.R[3 * k + 1] * bs[1] + X.R[3 * k + 2] * bs[2];
        nr |= (bs[3] >= 0.f) & (box_dist2(c, blo, bhi) <= bs[3] * bs[3]);
      }
    });
    return nr != 0;
  }

  // Exhaustive minimum signed distance over all sphere pairs (and the verdict), one lane.
  template <class Q>
  static __device__ __forceinline__ void min_signed_distance(const Q& q, const Consts& P, const CollConsts& K,
                                                             const float4* obs, bool& hit, float& minsd) {
    hit = false;
    minsd = __builtin_huge_valf();
    fk<float>(q, P.f, [&](auto J, const Rig<float>& X, const JP<float>&) {
      constexpr int l = decltype(J)::value;
      if constexpr (Topo::may_have_spheres(l)) narrow<true>(X, K, obs, l, 0, K.n_obs, hit, minsd);
    });
  }
};

}  // namespace mc
