// FP64 reference ("oracle") for the batched manifold projection of
// arXiv 2604.13323 (McVAMP). TEST INFRASTRUCTURE ONLY: it exists to check the
// HIP library, and only the tests, the package smoke check and the benchmark's
// CPU-baseline leg may load it. It shares no source with the HIP path and is
// deliberately built by different routes:
//   * the Jacobian comes from forward-mode dual numbers pushed through the
//     residual, not from analytic geometric columns;
//   * the Newton step is the minimum-norm solution of J dq = F obtained from a
//     Householder QR of J^T, not from a Cholesky factorisation of J J^T;
//   * the tangent projector of the VJP uses the same QR basis explicitly;
//   * singular values come from one-sided Jacobi SVD (Hestenes).
//
// What it computes (paper references):
//   ParallelProject + getDescentStep (Alg. 2, single stacked constraint block):
//     d <- F(q); stop when ||d|| < eps; step = alpha J^T (J J^T + lambda I)^-1 d;
//     optional divergence exit when ||step|| > MaxDistance; q <- q - step.
//   Pose error of Eq. 1 (TSR, T_w^0 = T_ref, grasp offset folded into the frame),
//   optionally with finite bounds B^w (Sec. III: a component inside its interval
//   contributes zero, outside it contributes its excess over the nearer bound),
//   relative pose error of Eq. 2, the humanoid constraints of the Digit
//   constraint figure (CoM equal to the support-polygon centroid, or the CoM
//   minus its nearest point of the support polygon, zero inside; closed-linkage
//   rod lengths), and the SO(3) log map with the first-order Taylor form of
//   1/sinc near zero (Sec. IV-A, the paragraph on the tracing compiler).
//   Scenes with rows that vanish on a region (bounded TSR components, the
//   polygon distance) have Jacobians of varying rank; there the step is the
//   pseudo-inverse solution J^+ F from a full SVD (one-sided Jacobi with the
//   right rotations accumulated), the plain definition of the minimum-norm step.
//   Collision check of the projected configurations (Sec. IV-A, the validation
//   that follows projection in the extend step): robot spheres vs obstacle
//   spheres, strict overlap ||c_i - o_j||^2 < (r_i + r_j)^2, brute force over
//   all pairs.
//   VJP (not in the paper): g_in = (I - J^+ J) g at the converged point.
//
// Readings where the paper is silent (also listed in the design notes):
//   per-configuration termination; iters = number of steps taken; the
//   convergence test is strict and uses the unweighted 2-norm of the stacked
//   residual; SINGULAR when sigma_min / sigma_max < 1e-12; DIVERGED is tested
//   before the update (the iterate is left unchanged).
//
// Build: g++ -O2 -fopenmp -shared -fPIC oracle.cpp -o liboracle.so
// (no intrinsics, no fast-math).

#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

// ------------------------------------------------------------------ scene
enum { B_POSE = 0, B_REL = 1, B_AXIS = 2, B_COM = 3, B_SPHERE = 4, B_LINEAR = 5, B_DIST = 6, B_HULL = 7 };
constexpr int kExt = 16;         // block data doubles of blob version 2
constexpr int kPoseBounded = 1;  // POSE block aux flag
enum { ST_CONVERGED = 0, ST_MAX_ITER = 1, ST_SINGULAR = 2, ST_DIVERGED = 3, ST_NONFINITE = 4 };

struct JointSpec { int parent, type, axis; double R[9], p[3]; };
struct FrameSpec { int link; double R[9], p[3]; };
struct BlockSpec { int type, fa, fb, mask, ref_from_qref, aux; double R[9], p[3], target[3], ext[kExt]; };
struct SphereSpec { int link; double c[3], r; };

struct Scene {
  int family = 0, d = 0, m = 0;
  std::vector<JointSpec> joints;
  std::vector<double> mass;
  std::vector<std::array<double, 3>> com;
  std::vector<FrameSpec> frames;
  std::vector<BlockSpec> blocks;
  std::vector<SphereSpec> spheres;
  std::vector<std::array<double, 4>> obstacles;
  std::vector<double> qref;
  std::vector<double> A, b;
};

struct Reader {
  const unsigned char* p; size_t n, off = 0; bool ok = true;
  template <class T> T get() {
    T v{};
    if (off + sizeof(T) > n) { ok = false; return v; }
    std::memcpy(&v, p + off, sizeof(T));
    off += sizeof(T);
    return v;
  }
  void getd(double* dst, int k) { for (int i = 0; i < k; ++i) dst[i] = get<double>(); }
};

int block_rows(const BlockSpec& b, const Scene& s) {
  switch (b.type) {
    case B_POSE: case B_REL: { int r = 0; for (int i = 0; i < 6; ++i) r += (b.mask >> i) & 1; return r; }
    case B_AXIS: case B_COM: case B_HULL: return 2;
    case B_SPHERE: case B_DIST: return 1;
    case B_LINEAR: return s.m;
  }
  return -1;
}

bool parse(const void* blob, size_t nbytes, Scene& s) {
  Reader r{static_cast<const unsigned char*>(blob), nbytes};
  int32_t h[16];
  for (int i = 0; i < 16; ++i) h[i] = r.get<int32_t>();
  if (!r.ok || h[0] != 0x5343434D || (h[1] != 1 && h[1] != 2)) return false;
  const bool v2 = h[1] == 2;
  s.family = h[2]; s.d = h[3]; s.m = h[4];
  int nj = h[5], nf = h[6], nb = h[7], ns = h[8], no = h[9], has_qref = h[10], has_lin = h[11];
  if (s.d <= 0 || s.m <= 0 || s.m > s.d || nj < 0 || nf < 0 || nb <= 0 || ns < 0 || no < 0) return false;
  s.joints.resize(nj);
  for (auto& j : s.joints) {
    j.parent = r.get<int32_t>(); j.type = r.get<int32_t>(); j.axis = r.get<int32_t>(); r.get<int32_t>();
    r.getd(j.R, 9); r.getd(j.p, 3);
  }
  s.mass.resize(nj); s.com.resize(nj);
  for (int k = 0; k < nj; ++k) { s.mass[k] = r.get<double>(); r.getd(s.com[k].data(), 3); }
  s.frames.resize(nf);
  for (auto& f : s.frames) { f.link = r.get<int32_t>(); r.get<int32_t>(); r.getd(f.R, 9); r.getd(f.p, 3); }
  s.blocks.resize(nb);
  for (auto& b : s.blocks) {
    b.type = r.get<int32_t>(); b.fa = r.get<int32_t>(); b.fb = r.get<int32_t>(); b.mask = r.get<int32_t>();
    b.ref_from_qref = r.get<int32_t>(); b.aux = r.get<int32_t>();
    r.getd(b.R, 9); r.getd(b.p, 3); r.getd(b.target, 3);
    for (int k = 0; k < kExt; ++k) b.ext[k] = 0.0;
    if (v2) r.getd(b.ext, kExt);
  }
  s.spheres.resize(ns);
  for (auto& sp : s.spheres) { sp.link = r.get<int32_t>(); r.get<int32_t>(); r.getd(sp.c, 3); sp.r = r.get<double>(); }
  s.obstacles.resize(no);
  for (auto& o : s.obstacles) r.getd(o.data(), 4);
  if (has_qref) { s.qref.resize(s.d); r.getd(s.qref.data(), s.d); }
  if (has_lin) { s.A.resize(size_t(s.m) * s.d); r.getd(s.A.data(), s.m * s.d); s.b.resize(s.m); r.getd(s.b.data(), s.m); }
  if (!r.ok) return false;
  // structural validation
  for (int j = 0; j < nj; ++j) {
    const auto& J = s.joints[j];
    if (J.parent < -1 || J.parent >= j || (J.type != 0 && J.type != 1) || J.axis < 0 || J.axis > 2) return false;
  }
  if (nj > 0 && nj != s.d) return false;
  int rows = 0;
  for (const auto& b : s.blocks) {
    int k = block_rows(b, s);
    if (k < 0) return false;
    if ((b.type == B_POSE || b.type == B_AXIS) && (b.fa < 0 || b.fa >= nf)) return false;
    if ((b.type == B_REL || b.type == B_DIST) && (b.fa < 0 || b.fa >= nf || b.fb < 0 || b.fb >= nf)) return false;
    if (b.type == B_POSE && (b.aux & kPoseBounded))
      for (int c = 0; c < 6; ++c) if (!(b.ext[c] <= b.ext[6 + c])) return false;
    if (b.type == B_HULL) {  // a convex polygon, counter-clockwise
      if (b.aux < 3 || b.aux > kExt / 2 || nj == 0) return false;
      for (int i = 0; i < b.aux; ++i) {
        const double* a = b.ext + 2 * i;
        const double* c = b.ext + 2 * ((i + 1) % b.aux);
        const double* e = b.ext + 2 * ((i + 2) % b.aux);
        if (!((c[0] - a[0]) * (e[1] - c[1]) - (c[1] - a[1]) * (e[0] - c[0]) > 0.0)) return false;
      }
    }
    if (b.ref_from_qref && !has_qref) return false;
    if (b.type == B_LINEAR && !has_lin) return false;
    if (b.type == B_SPHERE && s.d != 3) return false;
    rows += k;
  }
  if (rows != s.m) return false;
  for (const auto& f : s.frames) if (f.link < 0 || f.link >= nj) return false;
  for (const auto& sp : s.spheres) if (sp.link < -1 || sp.link >= nj) return false;
  return true;
}

// ------------------------------------------------------------ dual numbers
// Forward-mode AD value with one tangent direction, over any scalar T: Dn<double> gives first
// derivatives (the Jacobian), Dn<Dn<double>> second derivatives (the derivative of J along a
// direction, which differentiating the Newton iteration itself needs).
template <class T>
struct Dn {
  T v, d;
  Dn(double a = 0.0) : v(a), d(0.0) {}
  Dn(T a, T b) : v(a), d(b) {}
};
using Dual = Dn<double>;
template <class T> inline Dn<T> operator+(Dn<T> a, Dn<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> inline Dn<T> operator-(Dn<T> a, Dn<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> inline Dn<T> operator-(Dn<T> a) { return {-a.v, -a.d}; }
template <class T> inline Dn<T> operator*(Dn<T> a, Dn<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class T> inline Dn<T> operator/(Dn<T> a, Dn<T> b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
using std::sin; using std::cos; using std::sqrt; using std::atan2;
template <class T> inline Dn<T> sin(Dn<T> a) { return {sin(a.v), cos(a.v) * a.d}; }
template <class T> inline Dn<T> cos(Dn<T> a) { return {cos(a.v), -(sin(a.v) * a.d)}; }
template <class T> inline Dn<T> sqrt(Dn<T> a) { T s = sqrt(a.v); return {s, a.d / (T(2.0) * s)}; }
template <class T> inline Dn<T> atan2(Dn<T> y, Dn<T> x) {
  T r2 = x.v * x.v + y.v * y.v;
  return {atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / r2};
}
inline double val(double x) { return x; }
template <class T> inline double val(Dn<T> x) { return val(x.v); }

// ------------------------------------------------------- rigid transforms
template <class T> struct Tf { T R[3][3]; T p[3]; };

template <class T> Tf<T> tf_identity() {
  Tf<T> t;
  for (int i = 0; i < 3; ++i) { for (int k = 0; k < 3; ++k) t.R[i][k] = T(i == k ? 1.0 : 0.0); t.p[i] = T(0.0); }
  return t;
}
template <class T> Tf<T> tf_const(const double* R9, const double* p3) {
  Tf<T> t;
  for (int i = 0; i < 3; ++i) { for (int k = 0; k < 3; ++k) t.R[i][k] = T(R9[3 * i + k]); t.p[i] = T(p3[i]); }
  return t;
}
template <class T> Tf<T> tf_mul(const Tf<T>& a, const Tf<T>& b) {
  Tf<T> c;
  for (int i = 0; i < 3; ++i) {
    for (int k = 0; k < 3; ++k) c.R[i][k] = a.R[i][0] * b.R[0][k] + a.R[i][1] * b.R[1][k] + a.R[i][2] * b.R[2][k];
    c.p[i] = a.R[i][0] * b.p[0] + a.R[i][1] * b.p[1] + a.R[i][2] * b.p[2] + a.p[i];
  }
  return c;
}
template <class T> Tf<T> tf_inv(const Tf<T>& a) {
  Tf<T> c;
  for (int i = 0; i < 3; ++i) for (int k = 0; k < 3; ++k) c.R[i][k] = a.R[k][i];
  for (int i = 0; i < 3; ++i) c.p[i] = -(c.R[i][0] * a.p[0] + c.R[i][1] * a.p[1] + c.R[i][2] * a.p[2]);
  return c;
}
// Motion of one joint: rotation about (or translation along) a coordinate axis of its frame.
template <class T> Tf<T> joint_motion(int type, int axis, T x) {
  Tf<T> t = tf_identity<T>();
  if (type == 1) { t.p[axis] = x; return t; }
  T c = cos(x), s = sin(x);
  int i = (axis + 1) % 3, k = (axis + 2) % 3;  // rotation in the (i, k) plane
  t.R[i][i] = c; t.R[i][k] = -s;
  t.R[k][i] = s; t.R[k][k] = c;
  return t;
}

// Link frames T_j = T_parent(j) * O_j * Q_j(q_j).
template <class T> void forward_kinematics(const Scene& s, const T* q, std::vector<Tf<T>>& link) {
  const int nj = (int)s.joints.size();
  link.resize(nj);
  for (int j = 0; j < nj; ++j) {
    const auto& J = s.joints[j];
    Tf<T> base = J.parent < 0 ? tf_identity<T>() : link[J.parent];
    link[j] = tf_mul(tf_mul(base, tf_const<T>(J.R, J.p)), joint_motion<T>(J.type, J.axis, q[j]));
  }
}

template <class T> Tf<T> frame_pose(const Scene& s, const std::vector<Tf<T>>& link, int f) {
  return tf_mul(link[s.frames[f].link], tf_const<T>(s.frames[f].R, s.frames[f].p));
}

// SO(3) logarithm, vee form. v = vee(R - R^T)/2 = sin(theta) * axis, c = cos(theta).
// Near theta = 0 the factor theta / sin(theta) takes its first-order Taylor form 1 + s^2/6.
// theta (nullable) receives the rotation angle atan2(|v|, c) in [0, pi].
template <class T> void so3_log(const T R[3][3], T w[3], double* theta = nullptr) {
  T v[3] = {(R[2][1] - R[1][2]) * T(0.5), (R[0][2] - R[2][0]) * T(0.5), (R[1][0] - R[0][1]) * T(0.5)};
  T s2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  T c = (R[0][0] + R[1][1] + R[2][2] - T(1.0)) * T(0.5);
  T f;
  if (val(c) > 0.0 && val(s2) < 1e-8) {
    f = T(1.0) + s2 * T(1.0 / 6.0);
  } else {
    T s = sqrt(s2);
    f = atan2(s, c) / s;
  }
  for (int i = 0; i < 3; ++i) w[i] = f * v[i];
  if (theta) *theta = std::atan2(std::sqrt(val(s2)), val(c));
}

// Excess of a bounded component over its interval [lo, hi]: zero inside (a constant: no
// derivative), v - hi above it, v - lo below it (TSR bounds B^w, Sec. III).
template <class T> T bound_excess(T v, double lo, double hi) {
  if (val(v) > hi) return v - T(hi);
  if (val(v) < lo) return v - T(lo);
  return T(0.0);
}

// error rows [t; log(R)] of a pose error transform, selected by a 6-bit mask; max_theta (nullable)
// is raised to the error's rotation angle
template <class T> int pose_rows(const Tf<T>& e, int mask, T* out, double* max_theta = nullptr,
                                  const double* bounds = nullptr) {
  T w[3];
  double th = 0.0;
  so3_log(e.R, w, &th);
  if (max_theta && th > *max_theta) *max_theta = th;
  T all[6] = {e.p[0], e.p[1], e.p[2], w[0], w[1], w[2]};
  int r = 0;
  for (int i = 0; i < 6; ++i)
    if ((mask >> i) & 1) out[r++] = bounds ? bound_excess(all[i], bounds[i], bounds[6 + i]) : all[i];
  return r;
}

// Centre-of-mass xy of the robot: sum of m_l c_l over the links with mass, divided by their mass.
template <class T> void com_xy(const Scene& s, const std::vector<Tf<T>>& link, T* out) {
  T cx = T(0.0), cy = T(0.0);
  double M = 0.0;
  for (size_t l = 0; l < s.joints.size(); ++l) {
    double ml = s.mass[l];
    if (ml == 0.0) continue;
    const auto& L = link[l];
    const auto& c = s.com[l];
    T wx = L.R[0][0] * T(c[0]) + L.R[0][1] * T(c[1]) + L.R[0][2] * T(c[2]) + L.p[0];
    T wy = L.R[1][0] * T(c[0]) + L.R[1][1] * T(c[1]) + L.R[1][2] * T(c[2]) + L.p[1];
    cx = cx + T(ml) * wx;
    cy = cy + T(ml) * wy;
    M += ml;
  }
  out[0] = cx / T(M);
  out[1] = cy / T(M);
}

// Distance rows of a point x against a convex polygon V (nv counter-clockwise xy vertices): zero
// when x is inside or on the boundary, else x minus its nearest point of the boundary, found edge
// by edge (projection onto each edge's segment, the parameter clamped to its ends).
template <class T> void polygon_rows(const double* V, int nv, const T* x, T* out) {
  bool inside = true;
  for (int i = 0; i < nv; ++i) {
    const double* a = V + 2 * i;
    const double* b = V + 2 * ((i + 1) % nv);
    const double cr = (b[0] - a[0]) * (val(x[1]) - a[1]) - (b[1] - a[1]) * (val(x[0]) - a[0]);
    if (cr < 0.0) inside = false;
  }
  if (inside) { out[0] = T(0.0); out[1] = T(0.0); return; }
  double best = INFINITY;
  T nx = T(0.0), ny = T(0.0);
  for (int i = 0; i < nv; ++i) {
    const double* a = V + 2 * i;
    const double* b = V + 2 * ((i + 1) % nv);
    const double ex = b[0] - a[0], ey = b[1] - a[1];
    T t = ((x[0] - T(a[0])) * T(ex) + (x[1] - T(a[1])) * T(ey)) / T(ex * ex + ey * ey);
    if (val(t) < 0.0) t = T(0.0);
    if (val(t) > 1.0) t = T(1.0);
    const T cx = T(a[0]) + t * T(ex), cy = T(a[1]) + t * T(ey);
    const double dx = val(x[0]) - val(cx), dy = val(x[1]) - val(cy);
    if (dx * dx + dy * dy < best) { best = dx * dx + dy * dy; nx = cx; ny = cy; }
  }
  out[0] = x[0] - nx;
  out[1] = x[1] - ny;
}

// Targets of pose blocks (constant, FP64). For blocks flagged ref_from_qref the
// target is the pose (POSE) or relative pose (REL) at the reference configuration, and the
// rod length (DIST) the distance of its two frame origins there.
struct Targets { std::vector<Tf<double>> T; std::vector<double> L; };

Targets make_targets(const Scene& s) {
  Targets t;
  t.T.resize(s.blocks.size());
  t.L.assign(s.blocks.size(), 0.0);
  std::vector<Tf<double>> link;
  if (!s.qref.empty() && !s.joints.empty()) forward_kinematics<double>(s, s.qref.data(), link);
  for (size_t k = 0; k < s.blocks.size(); ++k) {
    const auto& b = s.blocks[k];
    if (b.ref_from_qref && b.type == B_POSE) t.T[k] = frame_pose(s, link, b.fa);
    else if (b.ref_from_qref && b.type == B_REL) t.T[k] = tf_mul(tf_inv(frame_pose(s, link, b.fa)), frame_pose(s, link, b.fb));
    else t.T[k] = tf_const<double>(b.R, b.p);
    if (b.type == B_DIST) {
      t.L[k] = b.target[0];
      if (b.ref_from_qref) {
        const Tf<double> pa = frame_pose(s, link, b.fa), pb = frame_pose(s, link, b.fb);
        double d2 = 0.0;
        for (int i = 0; i < 3; ++i) d2 += (pb.p[i] - pa.p[i]) * (pb.p[i] - pa.p[i]);
        t.L[k] = std::sqrt(d2);
      }
    }
  }
  return t;
}

// Stacked residual F(q) (rows in block order). max_theta (nullable) is raised to the largest
// rotation angle of the pose and relative-pose errors.
template <class T> void residual(const Scene& s, const Targets& tg, const T* q, T* F, double* max_theta = nullptr) {
  std::vector<Tf<T>> link;
  if (!s.joints.empty()) forward_kinematics<T>(s, q, link);
  int r = 0;
  for (size_t k = 0; k < s.blocks.size(); ++k) {
    const auto& b = s.blocks[k];
    Tf<T> Tref;
    for (int i = 0; i < 3; ++i) { for (int c = 0; c < 3; ++c) Tref.R[i][c] = T(tg.T[k].R[i][c]); Tref.p[i] = T(tg.T[k].p[i]); }
    switch (b.type) {
      case B_POSE: {  // Eq. 1: T_err = T_ref^-1 T_frame, minus the bounds B^w where the block has them
        const double* bnd = (b.aux & kPoseBounded) ? b.ext : nullptr;
        r += pose_rows(tf_mul(tf_inv(Tref), frame_pose(s, link, b.fa)), b.mask, F + r, max_theta, bnd);
        break;
      }
      case B_DIST: {  // closed linkage: distance of the two frame origins minus the rod length
        const Tf<T> pa = frame_pose(s, link, b.fa), pb = frame_pose(s, link, b.fb);
        T d2 = T(0.0);
        for (int i = 0; i < 3; ++i) d2 = d2 + (pb.p[i] - pa.p[i]) * (pb.p[i] - pa.p[i]);
        F[r++] = sqrt(d2) - T(tg.L[k]);
        break;
      }
      case B_HULL: {  // CoM xy minus its nearest point of the support polygon (zero inside)
        T x[2];
        com_xy(s, link, x);
        polygon_rows(b.ext, b.aux, x, F + r);
        r += 2;
        break;
      }
      case B_REL: {   // Eq. 2: T_err = T_ref^-1 (T_a^-1 T_b)
        Tf<T> rel = tf_mul(tf_inv(frame_pose(s, link, b.fa)), frame_pose(s, link, b.fb));
        r += pose_rows(tf_mul(tf_inv(Tref), rel), b.mask, F + r, max_theta);
        break;
      }
      case B_AXIS: {  // frame z-axis parallel to world z: x and y components of R e_z
        Tf<T> f = frame_pose(s, link, b.fa);
        F[r++] = f.R[0][2];
        F[r++] = f.R[1][2];
        break;
      }
      case B_COM: {   // centre of mass xy minus target
        T x[2];
        com_xy(s, link, x);
        F[r++] = x[0] - T(b.target[0]);
        F[r++] = x[1] - T(b.target[1]);
        break;
      }
      case B_SPHERE: {
        F[r++] = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] - T(1.0);
        break;
      }
      case B_LINEAR: {
        for (int i = 0; i < s.m; ++i) {
          T acc = T(-s.b[i]);
          for (int j = 0; j < s.d; ++j) acc = acc + T(s.A[size_t(i) * s.d + j]) * q[j];
          F[r++] = acc;
        }
        break;
      }
    }
  }
}

// Jacobian by forward-mode duals, one column per pass. J is m x d row-major. Over T = Dual the
// entries carry their own derivative along q's tangent.
template <class T>
void jacobian_t(const Scene& s, const Targets& tg, const T* q, T* J) {
  std::vector<Dn<T>> qd(s.d), Fd(s.m);
  for (int j = 0; j < s.d; ++j) {
    for (int i = 0; i < s.d; ++i) qd[i] = Dn<T>(q[i], T(i == j ? 1.0 : 0.0));
    residual<Dn<T>>(s, tg, qd.data(), Fd.data());
    for (int i = 0; i < s.m; ++i) J[size_t(i) * s.d + j] = Fd[i].d;
  }
}
void jacobian(const Scene& s, const Targets& tg, const double* q, double* J) { jacobian_t<double>(s, tg, q, J); }

// ------------------------------------------------------ dense linear algebra
// Householder QR of a rows x cols matrix A (column-major, rows >= cols), in place:
// R in the upper triangle, reflector vectors v_k (v_k[k] = 1 implied) below it, with tau.
void householder_qr(int rows, int cols, double* A, double* tau) {
  for (int k = 0; k < cols; ++k) {
    double* a = A + size_t(k) * rows;
    double nrm = 0.0;
    for (int i = k; i < rows; ++i) nrm += a[i] * a[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) { tau[k] = 0.0; continue; }
    double alpha = a[k] > 0 ? -nrm : nrm;  // new diagonal
    double v0 = a[k] - alpha;
    for (int i = k + 1; i < rows; ++i) a[i] /= v0;
    tau[k] = (alpha - a[k]) / alpha;        // = -v0 / alpha
    a[k] = alpha;
    for (int c = k + 1; c < cols; ++c) {
      double* b = A + size_t(c) * rows;
      double dot = b[k];
      for (int i = k + 1; i < rows; ++i) dot += a[i] * b[i];
      dot *= tau[k];
      b[k] -= dot;
      for (int i = k + 1; i < rows; ++i) b[i] -= dot * a[i];
    }
  }
}
// x <- H_k x with H_k = I - tau v v^T
void apply_reflector(int rows, int k, const double* A, const double* tau, double* x) {
  const double* a = A + size_t(k) * rows;
  double dot = x[k];
  for (int i = k + 1; i < rows; ++i) dot += a[i] * x[i];
  dot *= tau[k];
  x[k] -= dot;
  for (int i = k + 1; i < rows; ++i) x[i] -= dot * a[i];
}

// Singular values of a rows x cols matrix (column-major, rows >= cols), one-sided Jacobi.
void jacobi_singular_values(int rows, int cols, const double* A_in, double* sv) {
  std::vector<double> A(A_in, A_in + size_t(rows) * cols);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < cols - 1; ++p) {
      for (int r = p + 1; r < cols; ++r) {
        double* ap = A.data() + size_t(p) * rows;
        double* ar = A.data() + size_t(r) * rows;
        double alpha = 0, beta = 0, gamma = 0;
        for (int i = 0; i < rows; ++i) { alpha += ap[i] * ap[i]; beta += ar[i] * ar[i]; gamma += ap[i] * ar[i]; }
        if (gamma == 0.0) continue;
        double rel = std::fabs(gamma) / std::sqrt(alpha * beta);
        if (!(rel > 1e-15)) continue;
        off = std::max(off, rel);
        double zeta = (beta - alpha) / (2.0 * gamma);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < rows; ++i) {
          double x = ap[i], y = ar[i];
          ap[i] = c * x - sn * y;
          ar[i] = sn * x + c * y;
        }
      }
    }
    if (off < 1e-15) break;
  }
  for (int p = 0; p < cols; ++p) {
    double n = 0;
    for (int i = 0; i < rows; ++i) n += A[size_t(p) * rows + i] * A[size_t(p) * rows + i];
    sv[p] = std::sqrt(n);
  }
}

bool all_finite(const double* x, int n) { for (int i = 0; i < n; ++i) if (!std::isfinite(x[i])) return false; return true; }

struct Opts { double tol; int max_iter; double alpha, lambda, max_step; int mode; };  // mode 1: cyclic

// Descent step delta with J delta ~= F: minimum-norm (lambda = 0) or damped (lambda > 0).
// J is m x d row-major. Returns false on a singular Jacobian. smin_out (nullable) receives
// the smallest singular value of J.
bool descent_step(int m, int d, const double* J, const double* F, double lambda, double* delta,
                  double* smin_out = nullptr) {
  // singularity test on J (= on J^T) by its singular values
  std::vector<double> At(size_t(d) * m);  // J^T, column-major d x m: column i = row i of J
  for (int i = 0; i < m; ++i) for (int j = 0; j < d; ++j) At[size_t(i) * d + j] = J[size_t(i) * d + j];
  std::vector<double> sv(m);
  jacobi_singular_values(d, m, At.data(), sv.data());
  double smax = 0, smin = INFINITY;
  for (double x : sv) { smax = std::max(smax, x); smin = std::min(smin, x); }
  if (smin_out) *smin_out = smin;
  if (!(smax > 0.0) || smin / smax < 1e-12) return false;
  if (lambda <= 0.0) {
    // J^T = Q R. J delta = F  <=>  R^T (Q^T delta) = F; minimum-norm delta = Q z with R^T z = F.
    std::vector<double> tau(m);
    householder_qr(d, m, At.data(), tau.data());
    std::vector<double> z(d, 0.0);
    for (int i = 0; i < m; ++i) {
      double acc = F[i];
      for (int k = 0; k < i; ++k) acc -= At[size_t(i) * d + k] * z[k];  // R[k][i] = At[i*d + k]
      z[i] = acc / At[size_t(i) * d + i];
    }
    for (int k = m - 1; k >= 0; --k) apply_reflector(d, k, At.data(), tau.data(), z.data());
    for (int j = 0; j < d; ++j) delta[j] = z[j];
  } else {
    // minimise ||J delta - F||^2 + lambda ||delta||^2: least squares on [J; sqrt(lambda) I] delta = [F; 0]
    const int rows = m + d;
    std::vector<double> B(size_t(rows) * d, 0.0), rhs(rows, 0.0), tau(d);
    for (int j = 0; j < d; ++j) {
      for (int i = 0; i < m; ++i) B[size_t(j) * rows + i] = J[size_t(i) * d + j];
      B[size_t(j) * rows + m + j] = std::sqrt(lambda);
    }
    for (int i = 0; i < m; ++i) rhs[i] = F[i];
    householder_qr(rows, d, B.data(), tau.data());
    for (int k = 0; k < d; ++k) apply_reflector(rows, k, B.data(), tau.data(), rhs.data());
    for (int i = d - 1; i >= 0; --i) {
      double acc = rhs[i];
      for (int k = i + 1; k < d; ++k) acc -= B[size_t(k) * rows + i] * delta[k];
      delta[i] = acc / B[size_t(i) * rows + i];
    }
  }
  return true;
}

double norm2(const double* x, int n) { double a = 0; for (int i = 0; i < n; ++i) a += x[i] * x[i]; return std::sqrt(a); }

// Scenes whose rows vanish on a region (bounded TSR components, the polygon distance): the rank of
// J varies there, so the step is taken by pinv_step.
bool has_piecewise_rows(const Scene& s) {
  for (const auto& b : s.blocks)
    if (b.type == B_HULL || (b.type == B_POSE && (b.aux & kPoseBounded))) return true;
  return false;
}

constexpr double kRankCut = 1e-10;  // singular values at or below this fraction of the largest count as zero

// Full SVD of J (m x d row-major, m <= d) by one-sided Jacobi on J^T: the rotations that make the
// columns of A = J^T orthogonal are accumulated in V (m x m, column-major), so J^T V = A with
// orthogonal columns, sigma_k = ||A_k|| and J = V diag(sigma) U^T with U_k = A_k / sigma_k.
void jacobi_svd(int m, int d, const double* J, std::vector<double>& A, std::vector<double>& V, std::vector<double>& sv) {
  A.assign(size_t(d) * m, 0.0);
  V.assign(size_t(m) * m, 0.0);
  sv.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < d; ++j) A[size_t(i) * d + j] = J[size_t(i) * d + j];
    V[size_t(i) * m + i] = 1.0;
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < m - 1; ++p) {
      for (int r = p + 1; r < m; ++r) {
        double* ap = A.data() + size_t(p) * d;
        double* ar = A.data() + size_t(r) * d;
        double alpha = 0, beta = 0, gamma = 0;
        for (int i = 0; i < d; ++i) { alpha += ap[i] * ap[i]; beta += ar[i] * ar[i]; gamma += ap[i] * ar[i]; }
        if (gamma == 0.0 || alpha == 0.0 || beta == 0.0) continue;
        const double rel = std::fabs(gamma) / std::sqrt(alpha * beta);
        if (!(rel > 1e-15)) continue;
        off = std::max(off, rel);
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < d; ++i) {
          const double x = ap[i], y = ar[i];
          ap[i] = c * x - sn * y;
          ar[i] = sn * x + c * y;
        }
        double* vp = V.data() + size_t(p) * m;
        double* vr = V.data() + size_t(r) * m;
        for (int i = 0; i < m; ++i) {
          const double x = vp[i], y = vr[i];
          vp[i] = c * x - sn * y;
          vr[i] = sn * x + c * y;
        }
      }
    }
    if (off < 1e-15) break;
  }
  for (int k = 0; k < m; ++k) sv[k] = norm2(A.data() + size_t(k) * d, d);
}

// Pseudo-inverse step: delta = J^+ F (lambda = 0) or the damped J^T (J J^T + lambda I)^-1 F, from the
// SVD: delta = sum_k A_k (V_k^T F) / (sigma_k^2 + lambda) over the singular values above kRankCut
// sigma_max. Returns false when J = 0 while F is not. smin_out (nullable) receives the smallest
// singular value above the cut.
bool pinv_step(int m, int d, const double* J, const double* F, double lambda, double* delta, double* smin_out = nullptr) {
  std::vector<double> A, V, sv;
  jacobi_svd(m, d, J, A, V, sv);
  double smax = 0.0;
  for (double x : sv) smax = std::max(smax, x);
  for (int j = 0; j < d; ++j) delta[j] = 0.0;
  if (!(smax > 0.0)) {  // J = 0: no step; singular unless every row is zero too (a block all inside)
    if (smin_out) *smin_out = INFINITY;
    for (int i = 0; i < m; ++i) if (F[i] != 0.0) return false;
    return true;
  }
  double smin = INFINITY;
  for (int k = 0; k < m; ++k) {
    if (!(sv[k] > kRankCut * smax)) continue;
    smin = std::min(smin, sv[k]);
    double vf = 0.0;
    for (int i = 0; i < m; ++i) vf += V[size_t(k) * m + i] * F[i];
    const double c = vf / (sv[k] * sv[k] + lambda);
    for (int j = 0; j < d; ++j) delta[j] += A[size_t(k) * d + j] * c;
  }
  if (smin_out) *smin_out = smin;
  return true;
}

// g - P g with P the orthogonal projector onto the row space of J (the span of the U_k above the cut).
void pinv_tangent(int m, int d, const double* J, const double* g, double* out) {
  std::vector<double> A, V, sv;
  jacobi_svd(m, d, J, A, V, sv);
  double smax = 0.0;
  for (double x : sv) smax = std::max(smax, x);
  for (int j = 0; j < d; ++j) out[j] = g[j];
  for (int k = 0; k < m; ++k) {
    if (!(sv[k] > kRankCut * smax)) continue;
    const double* a = A.data() + size_t(k) * d;
    double ag = 0.0;
    for (int j = 0; j < d; ++j) ag += a[j] * g[j];
    const double c = ag / (sv[k] * sv[k]);
    for (int j = 0; j < d; ++j) out[j] -= a[j] * c;
  }
}


// ------------------------------------------------- the iteration as a differentiable map
// The same Householder QR and min-norm / damped step as above, over any scalar T, so the
// Newton iteration can run on dual numbers and carry the derivative of the projection map along.
template <class T>
void householder_qr_t(int rows, int cols, T* A, T* tau) {
  for (int k = 0; k < cols; ++k) {
    T* a = A + size_t(k) * rows;
    T nrm2 = T(0.0);
    for (int i = k; i < rows; ++i) nrm2 = nrm2 + a[i] * a[i];
    if (val(nrm2) == 0.0) { tau[k] = T(0.0); continue; }
    T nrm = sqrt(nrm2);
    T alpha = val(a[k]) > 0 ? -nrm : nrm;
    T v0 = a[k] - alpha;
    for (int i = k + 1; i < rows; ++i) a[i] = a[i] / v0;
    tau[k] = (alpha - a[k]) / alpha;
    a[k] = alpha;
    for (int c = k + 1; c < cols; ++c) {
      T* b = A + size_t(c) * rows;
      T dot = b[k];
      for (int i = k + 1; i < rows; ++i) dot = dot + a[i] * b[i];
      dot = dot * tau[k];
      b[k] = b[k] - dot;
      for (int i = k + 1; i < rows; ++i) b[i] = b[i] - dot * a[i];
    }
  }
}
template <class T>
void apply_reflector_t(int rows, int k, const T* A, const T* tau, T* x) {
  const T* a = A + size_t(k) * rows;
  T dot = x[k];
  for (int i = k + 1; i < rows; ++i) dot = dot + a[i] * x[i];
  dot = dot * tau[k];
  x[k] = x[k] - dot;
  for (int i = k + 1; i < rows; ++i) x[i] = x[i] - dot * a[i];
}
// delta with J delta = F (min-norm for lambda = 0, else the damped least-squares step); false when J
// is singular (the test on the values, as descent_step).
template <class T>
bool descent_step_t(int m, int d, const T* J, const T* F, double lambda, T* delta) {
  std::vector<double> Jv(size_t(m) * d), At(size_t(d) * m), sv(m);
  for (int i = 0; i < m * d; ++i) Jv[i] = val(J[i]);
  for (int i = 0; i < m; ++i) for (int j = 0; j < d; ++j) At[size_t(i) * d + j] = Jv[size_t(i) * d + j];
  jacobi_singular_values(d, m, At.data(), sv.data());
  double smax = 0, smin = INFINITY;
  for (double x : sv) { smax = std::max(smax, x); smin = std::min(smin, x); }
  if (!(smax > 0.0) || smin / smax < 1e-12) return false;
  if (lambda <= 0.0) {
    std::vector<T> B(size_t(d) * m), tau(m), z(d, T(0.0));
    for (int i = 0; i < m; ++i) for (int j = 0; j < d; ++j) B[size_t(i) * d + j] = J[size_t(i) * d + j];
    householder_qr_t(d, m, B.data(), tau.data());
    for (int i = 0; i < m; ++i) {
      T acc = F[i];
      for (int k = 0; k < i; ++k) acc = acc - B[size_t(i) * d + k] * z[k];
      z[i] = acc / B[size_t(i) * d + i];
    }
    for (int k = m - 1; k >= 0; --k) apply_reflector_t(d, k, B.data(), tau.data(), z.data());
    for (int j = 0; j < d; ++j) delta[j] = z[j];
  } else {
    const int rows = m + d;
    std::vector<T> B(size_t(rows) * d, T(0.0)), rhs(rows, T(0.0)), tau(d);
    for (int j = 0; j < d; ++j) {
      for (int i = 0; i < m; ++i) B[size_t(j) * rows + i] = J[size_t(i) * d + j];
      B[size_t(j) * rows + m + j] = T(std::sqrt(lambda));
    }
    for (int i = 0; i < m; ++i) rhs[i] = F[i];
    householder_qr_t(rows, d, B.data(), tau.data());
    for (int k = 0; k < d; ++k) apply_reflector_t(rows, k, B.data(), tau.data(), rhs.data());
    for (int i = d - 1; i >= 0; --i) {
      T acc = rhs[i];
      for (int k = i + 1; k < d; ++k) acc = acc - B[size_t(k) * rows + i] * delta[k];
      delta[i] = acc / B[size_t(i) * rows + i];
    }
  }
  return true;
}
// ParallelProject (Alg. 2, stacked) of one configuration, in place, over scalar T; the convergence and
// exit tests look at the values. After convergence `extra` more steps are taken (each is the identity
// on the values up to ||F||, and on the derivative the tangent projector: the converged map's
// derivative at an input that needs no step is that projector, not the identity). Returns the status;
// iters = steps taken before convergence.
template <class T>
int newton_map_t(const Scene& s, const Targets& tg, const Opts& o, T* q, int* iters, int extra = 0) {
  const int d = s.d, m = s.m;
  std::vector<T> F(m), J(size_t(m) * d), delta(d);
  int conv_at = -1;
  for (int k = 0;; ++k) {
    residual<T>(s, tg, q, F.data());
    double n2 = 0.0;
    bool fin = true;
    for (int i = 0; i < m; ++i) { n2 += val(F[i]) * val(F[i]); fin = fin && std::isfinite(val(F[i])); }
    if (conv_at < 0) *iters = k;
    if (!fin) return ST_NONFINITE;
    if (conv_at < 0 && std::sqrt(n2) < o.tol) conv_at = k;
    if (conv_at >= 0 && k - conv_at >= extra) return ST_CONVERGED;
    if (conv_at < 0 && k >= o.max_iter) return ST_MAX_ITER;
    jacobian_t<T>(s, tg, q, J.data());
    if (!descent_step_t<T>(m, d, J.data(), F.data(), o.lambda, delta.data())) return ST_SINGULAR;
    double s2 = 0.0;
    for (int j = 0; j < d; ++j) { delta[j] = delta[j] * T(o.alpha); s2 += val(delta[j]) * val(delta[j]); }
    if (!std::isfinite(s2)) return ST_NONFINITE;
    if (o.max_step > 0.0 && std::sqrt(s2) > o.max_step) return ST_DIVERGED;
    for (int j = 0; j < d; ++j) q[j] = q[j] - delta[j];
  }
}

// Path record of one projection (nullable), used by the parity tests to recognise outcomes that are
// not well posed for an exact comparison: [0] smallest sigma_min(J) over the steps taken, [1] longest
// step, [2] largest rotation angle of a pose error at any residual evaluation, [3] smallest
// multiplicative distance max(||F|| / tol, tol / ||F||) of a convergence test to the tolerance.
constexpr int kPathCols = 4;
void path_init(double* path) {
  if (!path) return;
  path[0] = INFINITY; path[1] = 0.0; path[2] = 0.0; path[3] = INFINITY;
}
void path_note_test(double* path, double nF, double tol, double theta) {
  if (!path) return;
  const double ratio = nF > tol ? nF / tol : tol / nF;  // +inf for nF = 0
  path[3] = std::min(path[3], ratio);
  path[2] = std::max(path[2], theta);
}

// Cyclic mode of ParallelProject (Alg. 2 with getDescentStep looping over the constraints,
// Sec. IV-C): each iteration first evaluates the whole stacked residual for the convergence
// test, then, for each constraint block in the scene's order, takes the min-norm step of that
// block's rows alone, evaluated at the configuration the previous blocks left. The divergence
// test applies to the displacement of the whole iteration (the step getDescentStep returns);
// when it fires the configuration is left where the iteration started.
void project_one_cyclic(const Scene& s, const Targets& tg, const Opts& o, const double* q0, double* q,
                        int8_t* status, int32_t* iters, double* resid, double* path) {
  const int d = s.d, m = s.m;
  const bool pw = has_piecewise_rows(s);
  std::vector<double> F(m), J(size_t(m) * d), delta(d), qs(d);
  for (int j = 0; j < d; ++j) q[j] = q0[j];
  path_init(path);
  for (int k = 0;; ++k) {
    double theta = 0.0;
    residual<double>(s, tg, q, F.data(), &theta);
    double nF = norm2(F.data(), m);
    path_note_test(path, nF, o.tol, theta);
    *resid = nF;
    *iters = k;
    if (!all_finite(F.data(), m) || !all_finite(q, d)) { *status = ST_NONFINITE; return; }
    if (nF < o.tol) { *status = ST_CONVERGED; return; }
    if (k >= o.max_iter) { *status = ST_MAX_ITER; return; }
    for (int j = 0; j < d; ++j) qs[j] = q[j];
    int r0 = 0;
    for (const auto& b : s.blocks) {
      const int mb = block_rows(b, s);
      double theta_b = 0.0;
      residual<double>(s, tg, q, F.data(), &theta_b);
      if (path) path[2] = std::max(path[2], theta_b);
      jacobian(s, tg, q, J.data());
      if (!all_finite(J.data() + size_t(r0) * d, mb * d)) { *status = ST_NONFINITE; return; }
      double smin = 0.0;
      const double* Jb = J.data() + size_t(r0) * d;
      const bool ok = pw ? pinv_step(mb, d, Jb, F.data() + r0, o.lambda, delta.data(), &smin)
                         : descent_step(mb, d, Jb, F.data() + r0, o.lambda, delta.data(), &smin);
      if (path) path[0] = std::min(path[0], smin);
      if (!ok) { *status = ST_SINGULAR; return; }
      for (int j = 0; j < d; ++j) delta[j] *= o.alpha;
      if (!all_finite(delta.data(), d)) { *status = ST_NONFINITE; return; }
      for (int j = 0; j < d; ++j) q[j] -= delta[j];
      r0 += mb;
    }
    double tot = 0.0;
    for (int j = 0; j < d; ++j) tot += (q[j] - qs[j]) * (q[j] - qs[j]);
    tot = std::sqrt(tot);
    if (path) path[1] = std::max(path[1], tot);
    if (o.max_step > 0.0 && tot > o.max_step) {
      for (int j = 0; j < d; ++j) q[j] = qs[j];
      *status = ST_DIVERGED;
      return;
    }
  }
}

// ParallelProject for one configuration (Alg. 2), per-configuration termination.
// path (nullable): the path record described at path_init.
void project_one(const Scene& s, const Targets& tg, const Opts& o, const double* q0, double* q,
                 int8_t* status, int32_t* iters, double* resid, double* path = nullptr) {
  const int d = s.d, m = s.m;
  const bool pw = has_piecewise_rows(s);
  std::vector<double> F(m), J(size_t(m) * d), delta(d);
  for (int j = 0; j < d; ++j) q[j] = q0[j];
  path_init(path);
  for (int k = 0;; ++k) {
    double theta = 0.0;
    residual<double>(s, tg, q, F.data(), &theta);
    double nF = norm2(F.data(), m);
    path_note_test(path, nF, o.tol, theta);
    *resid = nF;
    *iters = k;
    if (!all_finite(F.data(), m) || !all_finite(q, d)) { *status = ST_NONFINITE; return; }
    if (nF < o.tol) { *status = ST_CONVERGED; return; }
    if (k >= o.max_iter) { *status = ST_MAX_ITER; return; }
    jacobian(s, tg, q, J.data());
    if (!all_finite(J.data(), m * d)) { *status = ST_NONFINITE; return; }
    double smin = 0.0;
    const bool ok = pw ? pinv_step(m, d, J.data(), F.data(), o.lambda, delta.data(), &smin)
                       : descent_step(m, d, J.data(), F.data(), o.lambda, delta.data(), &smin);
    if (path) path[0] = std::min(path[0], smin);
    if (!ok) { *status = ST_SINGULAR; return; }
    for (int j = 0; j < d; ++j) delta[j] *= o.alpha;
    if (path) path[1] = std::max(path[1], norm2(delta.data(), d));
    if (!all_finite(delta.data(), d)) { *status = ST_NONFINITE; return; }
    if (o.max_step > 0.0 && norm2(delta.data(), d) > o.max_step) { *status = ST_DIVERGED; return; }
    for (int j = 0; j < d; ++j) q[j] -= delta[j];
  }
}

// World centres of the robot spheres at q (link -1: the configuration point itself).
void sphere_centres(const Scene& s, const double* q, std::vector<std::array<double, 3>>& c) {
  std::vector<Tf<double>> link;
  if (!s.joints.empty()) forward_kinematics<double>(s, q, link);
  c.resize(s.spheres.size());
  for (size_t i = 0; i < s.spheres.size(); ++i) {
    const auto& sp = s.spheres[i];
    if (sp.link < 0) { for (int a = 0; a < 3; ++a) c[i][a] = q[a] + sp.c[a]; continue; }
    const auto& L = link[sp.link];
    for (int a = 0; a < 3; ++a) c[i][a] = L.R[a][0] * sp.c[0] + L.R[a][1] * sp.c[1] + L.R[a][2] * sp.c[2] + L.p[a];
  }
}

void check_one(const Scene& s, const double* q, uint8_t* verdict, double* min_sd) {
  std::vector<std::array<double, 3>> c;
  sphere_centres(s, q, c);
  bool hit = false;
  double best = INFINITY;
  for (size_t i = 0; i < c.size(); ++i) {
    for (const auto& o : s.obstacles) {
      double dx = c[i][0] - o[0], dy = c[i][1] - o[1], dz = c[i][2] - o[2];
      double d2 = dx * dx + dy * dy + dz * dz;
      double rr = s.spheres[i].r + o[3];
      if (d2 < rr * rr) hit = true;
      best = std::min(best, std::sqrt(d2) - rr);
    }
  }
  *verdict = hit ? 1 : 0;
  if (min_sd) *min_sd = best;
}

int nthreads_or_default(int t) { return t > 0 ? t : omp_get_max_threads(); }

}  // namespace

// ================================================================ C ABI
extern "C" {

// info = {family, d, m, n_joints, n_frames, n_blocks, n_spheres, n_obstacles}
int oracle_scene_info(const void* blob, size_t nbytes, int32_t* info) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
  info[0] = s.family; info[1] = s.d; info[2] = s.m; info[3] = (int)s.joints.size(); info[4] = (int)s.frames.size();
  info[5] = (int)s.blocks.size(); info[6] = (int)s.spheres.size(); info[7] = (int)s.obstacles.size();
  return 0;
}

// Link frames at one configuration: out[n_joints][12] = R (row-major 9) then p (3).
int oracle_link_frames(const void* blob, size_t nbytes, const double* q, double* out) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
  std::vector<Tf<double>> link;
  forward_kinematics<double>(s, q, link);
  for (size_t j = 0; j < link.size(); ++j) {
    for (int i = 0; i < 3; ++i) for (int k = 0; k < 3; ++k) out[12 * j + 3 * i + k] = link[j].R[i][k];
    for (int i = 0; i < 3; ++i) out[12 * j + 9 + i] = link[j].p[i];
  }
  return 0;
}

// End-effector frame poses at one configuration: out[n_frames][12].
int oracle_frame_poses(const void* blob, size_t nbytes, const double* q, double* out) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
  std::vector<Tf<double>> link;
  forward_kinematics<double>(s, q, link);
  for (size_t f = 0; f < s.frames.size(); ++f) {
    Tf<double> t = frame_pose(s, link, (int)f);
    for (int i = 0; i < 3; ++i) for (int k = 0; k < 3; ++k) out[12 * f + 3 * i + k] = t.R[i][k];
    for (int i = 0; i < 3; ++i) out[12 * f + 9 + i] = t.p[i];
  }
  return 0;
}

// SO(3) log of one rotation matrix (row-major), for the log/exp identity pin.
void oracle_so3_log(const double* R9, double* w) {
  double R[3][3];
  for (int i = 0; i < 3; ++i) for (int k = 0; k < 3; ++k) R[i][k] = R9[3 * i + k];
  so3_log<double>(R, w);
}

// F for n configurations, q row-major [n][d], F [n][m].
int oracle_residual(const void* blob, size_t nbytes, int64_t n, const double* q, double* F, int nthreads) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
  Targets tg = make_targets(s);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads))
  for (int64_t i = 0; i < n; ++i) residual<double>(s, tg, q + i * s.d, F + i * s.m);
  return 0;
}

// J for n configurations: [n][m][d].
int oracle_jacobian(const void* blob, size_t nbytes, int64_t n, const double* q, double* J, int nthreads) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
  Targets tg = make_targets(s);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads))
  for (int64_t i = 0; i < n; ++i) jacobian(s, tg, q + i * s.d, J + i * size_t(s.m) * s.d);
  return 0;
}

// Projection of n configurations (row-major [n][d]).
// path_info (nullable) [n][4]: the path record described at path_init.
// mode 0: stacked system per step; mode 1: cyclic over the constraint blocks.
int oracle_project(const void* blob, size_t nbytes, int64_t n, const double* q_in, double* q_out,
                   int8_t* status, int32_t* iters, double* resid, double tol, int32_t max_iter,
                   double alpha, double lambda, double max_step, int nthreads, double* path_info, int mode) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
  if (n < 0 || !(tol > 0) || max_iter < 0 || (mode != 0 && mode != 1)) return 2;
  Targets tg = make_targets(s);
  Opts o{tol, max_iter, alpha, lambda, max_step, mode};
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads_or_default(nthreads))
  for (int64_t i = 0; i < n; ++i) {
    double* pi = path_info ? path_info + kPathCols * i : nullptr;
    if (mode == 1)
      project_one_cyclic(s, tg, o, q_in + i * s.d, q_out + i * s.d, status + i, iters + i, resid + i, pi);
    else
      project_one(s, tg, o, q_in + i * s.d, q_out + i * s.d, status + i, iters + i, resid + i, pi);
  }
  return 0;
}

// Collision verdicts (0 free, 1 collision) and minimum signed distance, brute force over all pairs.
int oracle_check(const void* blob, size_t nbytes, int64_t n, const double* q, uint8_t* verdict,
                 double* min_sd, int nthreads) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads))
  for (int64_t i = 0; i < n; ++i) check_one(s, q + i * s.d, verdict + i, min_sd ? min_sd + i : nullptr);
  return 0;
}

// VJP through the converged projection: g_in = g - Q Q^T g with J(q*)^T = Q R.
// Also returns kappa2(J J^T) = (sigma_max / sigma_min)^2. Configurations whose status is not
// CONVERGED get g_in = 0 and kappa = NaN.
int oracle_vjp(const void* blob, size_t nbytes, int64_t n, const double* q, const int8_t* status,
               const double* g, double* g_in, double* kappa, int nthreads) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
  Targets tg = make_targets(s);
  const int d = s.d, m = s.m;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads))
  for (int64_t c = 0; c < n; ++c) {
    double* out = g_in + c * d;
    if (status && status[c] != ST_CONVERGED) {
      for (int j = 0; j < d; ++j) out[j] = 0.0;
      if (kappa) kappa[c] = NAN;
      continue;
    }
    std::vector<double> J(size_t(m) * d), At(size_t(d) * m), tau(m), w(d), sv(m);
    jacobian(s, tg, q + c * d, J.data());
    if (has_piecewise_rows(s)) {  // rank varies: the projector from the SVD, no condition number
      pinv_tangent(m, d, J.data(), g + c * d, out);
      if (kappa) kappa[c] = NAN;
      continue;
    }
    for (int i = 0; i < m; ++i) for (int j = 0; j < d; ++j) At[size_t(i) * d + j] = J[size_t(i) * d + j];
    jacobi_singular_values(d, m, At.data(), sv.data());
    double smax = 0, smin = INFINITY;
    for (double x : sv) { smax = std::max(smax, x); smin = std::min(smin, x); }
    if (kappa) kappa[c] = (smax / smin) * (smax / smin);
    householder_qr(d, m, At.data(), tau.data());
    const double* gc = g + c * d;
    for (int j = 0; j < d; ++j) w[j] = gc[j];
    for (int k = 0; k < m; ++k) apply_reflector(d, k, At.data(), tau.data(), w.data());  // w = Q_full^T g
    for (int j = m; j < d; ++j) w[j] = 0.0;                                              // keep Q^T g
    for (int k = m - 1; k >= 0; --k) apply_reflector(d, k, At.data(), tau.data(), w.data());  // w = Q Q^T g
    for (int j = 0; j < d; ++j) out[j] = gc[j] - w[j];
  }
  return 0;
}

// Condition estimate of J J^T + lambda I that decides the FP32 -> FP64 switch: the Cholesky factor
// L (textbook row-by-row algorithm, FP64) gives kappa_est = (max L_ii / min L_ii)^2, a lower bound
// of the spectral condition number; kappa_est = +inf when a pivot is not positive. kappa2 (nullable)
// receives (sigma_max / sigma_min)^2 of J from the singular values.
int oracle_kappa_est(const void* blob, size_t nbytes, int64_t n, const double* q, double lambda, double* kappa_est,
                     double* kappa2, int nthreads) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
  Targets tg = make_targets(s);
  const int d = s.d, m = s.m;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_or_default(nthreads))
  for (int64_t c = 0; c < n; ++c) {
    std::vector<double> J(size_t(m) * d), G(size_t(m) * m, 0.0), L(size_t(m) * m, 0.0);
    jacobian(s, tg, q + c * d, J.data());
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < m; ++k) {
        double acc = i == k ? lambda : 0.0;
        for (int j = 0; j < d; ++j) acc += J[size_t(i) * d + j] * J[size_t(k) * d + j];
        G[size_t(i) * m + k] = acc;
      }
    bool ok = true;
    double lmin = INFINITY, lmax = 0.0;
    for (int i = 0; i < m && ok; ++i) {
      for (int k = 0; k <= i; ++k) {
        double acc = G[size_t(i) * m + k];
        for (int j = 0; j < k; ++j) acc -= L[size_t(i) * m + j] * L[size_t(k) * m + j];
        if (i == k) {
          if (!(acc > 0.0)) { ok = false; break; }
          L[size_t(i) * m + i] = std::sqrt(acc);
          lmin = std::min(lmin, L[size_t(i) * m + i]);
          lmax = std::max(lmax, L[size_t(i) * m + i]);
        } else {
          L[size_t(i) * m + k] = acc / L[size_t(k) * m + k];
        }
      }
    }
    kappa_est[c] = ok ? (lmax / lmin) * (lmax / lmin) : INFINITY;
    if (kappa2) {
      std::vector<double> At(size_t(d) * m), sv(m);
      for (int i = 0; i < m; ++i) for (int j = 0; j < d; ++j) At[size_t(i) * d + j] = J[size_t(i) * d + j];
      jacobi_singular_values(d, m, At.data(), sv.data());
      double smax = 0, smin = INFINITY;
      for (double x : sv) { smax = std::max(smax, x); smin = std::min(smin, x); }
      kappa2[c] = (smax / smin) * (smax / smin);
    }
  }
  return 0;
}

// Exact VJP of the projection map q0 -> P(q0) at arbitrary (off-manifold) inputs: the Jacobian of
// the map is obtained column by column by running the Newton iteration on dual numbers seeded
// with the input direction e_i (forward-mode through every step, second derivatives of F
// included), to the given tolerance and one step past it; g_in = (dP/dq0)^T g. Run to a tight
// tolerance (1e-13 or below) this is the derivative of the fully converged projection (up to
// the final ||F||). status [n] receives the value iteration's status; configurations that do not
// converge get g_in = 0.
int oracle_vjp_exact(const void* blob, size_t nbytes, int64_t n, const double* q0, const double* g, double* g_in,
                     double tol, int32_t max_iter, double alpha, double lambda, int8_t* status, int nthreads) {
  Scene s;
  if (!parse(blob, nbytes, s)) return 1;
  if (n < 0 || !(tol > 0) || max_iter < 0) return 2;
  if (has_piecewise_rows(s)) return 3;  // the dual-number step is the QR one, which needs full row rank
  Targets tg = make_targets(s);
  const int d = s.d;
  Opts o{tol, max_iter, alpha, lambda, 0.0, 0};
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_or_default(nthreads))
  for (int64_t c = 0; c < n; ++c) {
    std::vector<Dual> q(d);
    double* out = g_in + c * d;
    int st = ST_CONVERGED, it = 0;
    for (int i = 0; i < d && st == ST_CONVERGED; ++i) {
      for (int j = 0; j < d; ++j) q[j] = Dual(q0[c * d + j], j == i ? 1.0 : 0.0);
      st = newton_map_t<Dual>(s, tg, o, q.data(), &it, 1);
      double acc = 0.0;
      for (int j = 0; j < d; ++j) acc += q[j].d * g[c * d + j];  // (dP_j / dq0_i) g_j
      out[i] = acc;
    }
    if (status) status[c] = int8_t(st);
    if (st != ST_CONVERGED)
      for (int i = 0; i < d; ++i) out[i] = 0.0;
  }
  return 0;
}

// Path-length loss over geodesics (CSR offsets) and its gradient with respect to every point.
// L = sum_g sum_i ||q_{i+1} - q_i||; dL/dq_i = u_{i-1} - u_i with u = delta / max(||delta||, 1e-12).
int oracle_path_length(int64_t n, int32_t d, const double* q, const int32_t* offs, int32_t n_geo,
                       double* grad, double* loss) {
  for (int64_t i = 0; i < n * d; ++i) grad[i] = 0.0;
  double L = 0.0;
  std::vector<double> u(d);
  for (int g = 0; g < n_geo; ++g) {
    for (int i = offs[g]; i + 1 < offs[g + 1]; ++i) {
      double nn = 0.0;
      for (int j = 0; j < d; ++j) { u[j] = q[size_t(i + 1) * d + j] - q[size_t(i) * d + j]; nn += u[j] * u[j]; }
      nn = std::sqrt(nn);
      L += nn;
      double inv = 1.0 / std::max(nn, 1e-12);
      for (int j = 0; j < d; ++j) {
        grad[size_t(i) * d + j] -= u[j] * inv;
        grad[size_t(i + 1) * d + j] += u[j] * inv;
      }
    }
  }
  *loss = L;
  return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
