// C-ABI of the mcproj library: problem lifecycle, argument validation, dispatch of the
// per-family kernels, and the small utility kernels (work-queue reset, geodesic
// interpolation, path-length gradient, per-geodesic success flags).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mcproj.h"
#include "kin.hpp"
#include "ops.hpp"

using namespace mc;

namespace {

thread_local std::string g_err;

mc_status fail(mc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
mc_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? MC_ERR_OOM : MC_ERR_HIP;
}

// ------------------------------------------------------------------ host scene
struct HJoint { int parent, type, axis; double R[9], p[3]; };
struct HFrame { int link; double R[9], p[3]; };
struct HBlock { int type, fa, fb, mask, ref_from_qref, aux; double R[9], p[3], target[3], ext[16]; };
struct HSphere { int link; double c[3], r; };
struct HScene {
  int family = 0, d = 0, m = 0;
  std::vector<HJoint> joints;
  std::vector<double> mass;
  std::vector<std::array<double, 3>> com;
  std::vector<HFrame> frames;
  std::vector<HBlock> blocks;
  std::vector<HSphere> spheres;
  std::vector<std::array<double, 4>> obs;
  std::vector<double> qref, A, b;
};

struct Cursor {
  const unsigned char* p;
  size_t n, off = 0;
  bool ok = true;
  template <class T> T get() {
    T v{};
    if (off + sizeof(T) > n) { ok = false; return v; }
    std::memcpy(&v, p + off, sizeof(T));
    off += sizeof(T);
    return v;
  }
  void getd(double* d, int k) { for (int i = 0; i < k; ++i) d[i] = get<double>(); }
};

bool parse_blob(const void* blob, size_t nbytes, HScene& s, std::string& err) {
  Cursor c{static_cast<const unsigned char*>(blob), nbytes};
  int32_t h[16];
  for (int i = 0; i < 16; ++i) h[i] = c.get<int32_t>();
  if (!c.ok || h[0] != 0x5343434D) { err = "scene blob: bad magic or truncated header"; return false; }
  if (h[1] != 1 && h[1] != 2) { err = "scene blob: unsupported version"; return false; }
  const bool v2 = h[1] == 2;  // every block record is followed by 16 doubles of block data
  s.family = h[2]; s.d = h[3]; s.m = h[4];
  const int nj = h[5], nf = h[6], nb = h[7], ns = h[8], no = h[9], has_qref = h[10], has_lin = h[11];
  if (s.d <= 0 || s.m <= 0 || nj < 0 || nf < 0 || nb <= 0 || ns < 0 || no < 0 || nj > 4096 || nf > 4096 ||
      nb > 4096 || ns > 1 << 20 || no > 1 << 24 || s.d > 4096 || s.m > 4096) {
    err = "scene blob: bad counts"; return false;
  }
  s.joints.resize(nj);
  for (auto& j : s.joints) {
    j.parent = c.get<int32_t>(); j.type = c.get<int32_t>(); j.axis = c.get<int32_t>(); c.get<int32_t>();
    c.getd(j.R, 9); c.getd(j.p, 3);
  }
  s.mass.resize(nj); s.com.resize(nj);
  for (int k = 0; k < nj; ++k) { s.mass[k] = c.get<double>(); c.getd(s.com[k].data(), 3); }
  s.frames.resize(nf);
  for (auto& f : s.frames) { f.link = c.get<int32_t>(); c.get<int32_t>(); c.getd(f.R, 9); c.getd(f.p, 3); }
  s.blocks.resize(nb);
  for (auto& b : s.blocks) {
    b.type = c.get<int32_t>(); b.fa = c.get<int32_t>(); b.fb = c.get<int32_t>(); b.mask = c.get<int32_t>();
    b.ref_from_qref = c.get<int32_t>(); b.aux = c.get<int32_t>();
    c.getd(b.R, 9); c.getd(b.p, 3); c.getd(b.target, 3);
    for (int k = 0; k < 16; ++k) b.ext[k] = 0.0;
    if (v2) c.getd(b.ext, 16);
  }
  s.spheres.resize(ns);
  for (auto& sp : s.spheres) { sp.link = c.get<int32_t>(); c.get<int32_t>(); c.getd(sp.c, 3); sp.r = c.get<double>(); }
  s.obs.resize(no);
  for (auto& o : s.obs) c.getd(o.data(), 4);
  if (has_qref) { s.qref.resize(s.d); c.getd(s.qref.data(), s.d); }
  if (has_lin) { s.A.resize(size_t(s.m) * s.d); c.getd(s.A.data(), s.m * s.d); s.b.resize(s.m); c.getd(s.b.data(), s.m); }
  if (!c.ok) { err = "scene blob: truncated"; return false; }
  for (int j = 0; j < nj; ++j) {
    const auto& J = s.joints[j];
    if (J.parent < -1 || J.parent >= j || (J.type != 0 && J.type != 1) || J.axis < 0 || J.axis > 2) {
      err = "scene blob: bad joint " + std::to_string(j); return false;
    }
  }
  for (const auto& f : s.frames) if (f.link < 0 || f.link >= nj) { err = "scene blob: bad frame link"; return false; }
  for (const auto& sp : s.spheres) if (sp.link < -1 || sp.link >= nj || !(sp.r >= 0)) { err = "scene blob: bad sphere"; return false; }
  for (const auto& o : s.obs) if (!(o[3] >= 0) || !std::isfinite(o[0] + o[1] + o[2])) { err = "scene blob: bad obstacle"; return false; }
  for (const auto& b : s.blocks) if (b.ref_from_qref && !has_qref) { err = "scene blob: block needs q_ref"; return false; }
  return true;
}

// ---- host forward kinematics (reference poses at q_ref, at create time only)
struct HT { double R[9], p[3]; };
HT ht_mul(const HT& a, const HT& b) {
  HT c;
  for (int i = 0; i < 3; ++i) {
    for (int k = 0; k < 3; ++k) c.R[3 * i + k] = a.R[3 * i] * b.R[k] + a.R[3 * i + 1] * b.R[3 + k] + a.R[3 * i + 2] * b.R[6 + k];
    c.p[i] = a.R[3 * i] * b.p[0] + a.R[3 * i + 1] * b.p[1] + a.R[3 * i + 2] * b.p[2] + a.p[i];
  }
  return c;
}
HT ht_inv(const HT& a) {
  HT c;
  for (int i = 0; i < 3; ++i) for (int k = 0; k < 3; ++k) c.R[3 * i + k] = a.R[3 * k + i];
  for (int i = 0; i < 3; ++i) c.p[i] = -(c.R[3 * i] * a.p[0] + c.R[3 * i + 1] * a.p[1] + c.R[3 * i + 2] * a.p[2]);
  return c;
}
HT ht_make(const double* R, const double* p) {
  HT t;
  std::memcpy(t.R, R, sizeof t.R);
  std::memcpy(t.p, p, sizeof t.p);
  return t;
}
std::vector<HT> host_fk(const HScene& s, const double* q) {
  std::vector<HT> L(s.joints.size());
  for (size_t j = 0; j < s.joints.size(); ++j) {
    const auto& J = s.joints[j];
    HT base;
    if (J.parent < 0) {
      for (int k = 0; k < 9; ++k) base.R[k] = (k % 4 == 0) ? 1.0 : 0.0;
      base.p[0] = base.p[1] = base.p[2] = 0.0;
    } else {
      base = L[J.parent];
    }
    HT t = ht_mul(base, ht_make(J.R, J.p));
    HT m;
    for (int k = 0; k < 9; ++k) m.R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    m.p[0] = m.p[1] = m.p[2] = 0.0;
    if (J.type == 1) {
      m.p[J.axis] = q[j];
    } else {
      const double c = std::cos(q[j]), sn = std::sin(q[j]);
      const int i = (J.axis + 1) % 3, k = (J.axis + 2) % 3;
      m.R[3 * i + i] = c; m.R[3 * i + k] = -sn; m.R[3 * k + i] = sn; m.R[3 * k + k] = c;
    }
    L[j] = ht_mul(t, m);
  }
  return L;
}

// ---- compiled-structure check
bool is_identity(const double* R) {
  for (int k = 0; k < 9; ++k)
    if (std::fabs(R[k] - ((k % 4 == 0) ? 1.0 : 0.0)) > 1e-12) return false;
  return true;
}

template <class Topo>
bool matches_topology(const HScene& s, std::string& err) {
  using KI = KInfo<Topo>;
  if ((int)s.joints.size() != Topo::NJ || s.d != Topo::NJ) { err = "joint count does not match the compiled family"; return false; }
  if (s.m != Topo::M) { err = "row count does not match the compiled family"; return false; }
  for (int j = 0; j < Topo::NJ; ++j) {
    if (s.joints[j].parent != Topo::parent[j] || s.joints[j].type != Topo::jtype[j] || s.joints[j].axis != Topo::axis[j]) {
      err = "joint " + std::to_string(j) + " does not match the compiled family"; return false;
    }
    if (!Topo::origin_rot && !is_identity(s.joints[j].R)) { err = "family expects pure-translation joint origins"; return false; }
    if (Topo::has_com && Topo::massless(j) && (s.mass[j] != 0.0)) {
      err = "family expects massless link " + std::to_string(j);
      return false;
    }
  }
  if ((int)s.frames.size() != Topo::NF) { err = "frame count does not match the compiled family"; return false; }
  for (int f = 0; f < Topo::NF; ++f) {
    if (s.frames[f].link != Topo::frame_link[f]) { err = "frame link does not match the compiled family"; return false; }
    if (!Topo::frame_rot && !is_identity(s.frames[f].R)) { err = "family expects pure-translation frame offsets"; return false; }
  }
  if ((int)s.blocks.size() != Topo::NB) { err = "block count does not match the compiled family"; return false; }
  for (int b = 0; b < Topo::NB; ++b) {
    const auto& B = s.blocks[b];
    if (B.type != Topo::btype[b]) { err = "block type does not match the compiled family"; return false; }
    if ((B.type == B_POSE || B.type == B_REL || B.type == B_AXIS) && B.fa != Topo::bfa[b]) { err = "block frame mismatch"; return false; }
    if (B.type == B_REL && B.fb != Topo::bfb[b]) { err = "block frame mismatch"; return false; }
    if ((B.type == B_POSE || B.type == B_REL) && B.mask != Topo::bmask[b]) { err = "block row mask mismatch"; return false; }
    if ((B.type == B_COM || B.type == B_HULL) && !Topo::has_com) { err = "unexpected CoM block"; return false; }
    if (B.type == B_DIST && (B.fa != Topo::bfa[b] || B.fb != Topo::bfb[b])) { err = "block frame mismatch"; return false; }
    if (B.type == B_POSE) {
      if ((B.aux & BF_BOUNDED) != (Topo::bflags[b] & BF_BOUNDED)) { err = "pose block bounds flag mismatch"; return false; }
      if (B.aux & BF_BOUNDED)
        for (int c = 0; c < 6; ++c)
          if (!(B.ext[c] <= B.ext[6 + c])) { err = "pose block bounds: lo > hi or NaN"; return false; }
    }
    if (B.type == B_HULL) {  // a convex polygon given counter-clockwise, 3 to MAXHV vertices
      if (B.aux < 3 || B.aux > MAXHV) { err = "support polygon: 3 to 8 vertices"; return false; }
      for (int i = 0; i < B.aux; ++i) {
        const double* a = B.ext + 2 * i;
        const double* c = B.ext + 2 * ((i + 1) % B.aux);
        const double* e = B.ext + 2 * ((i + 2) % B.aux);
        if (!((c[0] - a[0]) * (e[1] - c[1]) - (c[1] - a[1]) * (e[0] - c[0]) > 0.0)) {
          err = "support polygon: not convex and counter-clockwise"; return false;
        }
      }
    }
  }
  for (const auto& sp : s.spheres)
    if (sp.link < 0 || !Topo::may_have_spheres(sp.link)) { err = "sphere on a link without geometry slot"; return false; }
  (void)sizeof(KI);
  return true;
}

const FamilyOps* ops_for(int family, int f64) {
  switch (family) {
    case MC_FAMILY_SPHERE: return f64 ? &ops_sphere3_f64 : &ops_sphere3_f32;
    case MC_FAMILY_LINEAR: return f64 ? &ops_linear_f64 : &ops_linear_f32;
    case MC_FAMILY_PLANAR2: return f64 ? &ops_planar2_f64 : &ops_planar2_f32;
    case MC_FAMILY_ARM7_AXIS: return f64 ? &ops_arm7_axis_f64 : &ops_arm7_axis_f32;
    case MC_FAMILY_DUAL14_REL: return f64 ? &ops_dual14_rel_f64 : &ops_dual14_rel_f32;
    case MC_FAMILY_HUMANOID36: return f64 ? &ops_humanoid36_f64 : &ops_humanoid36_f32;
    case MC_FAMILY_DIGIT36: return f64 ? &ops_digit36_f64 : &ops_digit36_f32;
    case MC_FAMILY_ARM7_TSR: return f64 ? &ops_arm7_tsr_f64 : &ops_arm7_tsr_f32;
  }
  return nullptr;
}

bool validate_family(const HScene& s, std::string& err) {
  switch (s.family) {
    case MC_FAMILY_SPHERE:
      if (s.d != 3 || s.m != 1 || !s.joints.empty() || s.blocks.size() != 1 || s.blocks[0].type != B_SPHERE) {
        err = "sphere family: expects d = 3, m = 1, one SPHERE block, no joints"; return false;
      }
      if (s.spheres.size() > 1 || (s.spheres.size() == 1 && s.spheres[0].link != -1)) {
        err = "sphere family: at most one point-robot sphere (link -1)"; return false;
      }
      return true;
    case MC_FAMILY_LINEAR:
      if (s.d > LIN_D || s.m > LIN_M || s.m > s.d || !s.joints.empty() || s.blocks.size() != 1 ||
          s.blocks[0].type != B_LINEAR || s.A.empty() || !s.spheres.empty()) {
        err = "linear family: expects d <= 8, m <= min(6, d), one LINEAR block, no joints or spheres"; return false;
      }
      return true;
    case MC_FAMILY_PLANAR2: return matches_topology<TopoPlanar2>(s, err);
    case MC_FAMILY_ARM7_AXIS: return matches_topology<TopoArm7Axis>(s, err);
    case MC_FAMILY_DUAL14_REL: return matches_topology<TopoDual14Rel>(s, err);
    case MC_FAMILY_HUMANOID36: return matches_topology<TopoHumanoid36>(s, err);
    case MC_FAMILY_DIGIT36: return matches_topology<TopoDigit36>(s, err);
    case MC_FAMILY_ARM7_TSR: return matches_topology<TopoArm7Tsr>(s, err);
  }
  err = "unknown scene family " + std::to_string(s.family);
  return false;
}

// ---- obstacle clusters: recursive median split on the widest axis, <= kClusterSize each
constexpr int kClusterSize = 16;
constexpr double kBoundMargin = 1e-4;  // metres added to every bound (covers FP32 rounding)
// exact-check tail grid: workgroups of 256 per CU (its short-queue path takes up to 4 waves' work
// items per workgroup)
constexpr int kCheckTailBlocksPerCu = 4;
constexpr int kGroupSize = 8;          // clusters per group (the second level of boxes)
static_assert((MAXC + kGroupSize - 1) / kGroupSize <= MAXSUP, "group table too small");

void build_clusters(std::vector<std::array<double, 4>>& obs, int lo, int hi,
                    std::vector<std::array<double, 4>>& cl, std::vector<std::array<int, 2>>& rg) {
  if (hi - lo <= kClusterSize) {
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int i = lo; i < hi; ++i)
      for (int a = 0; a < 3; ++a) { mn[a] = std::min(mn[a], obs[i][a]); mx[a] = std::max(mx[a], obs[i][a]); }
    std::array<double, 4> c{0.5 * (mn[0] + mx[0]), 0.5 * (mn[1] + mx[1]), 0.5 * (mn[2] + mx[2]), 0.0};
    for (int i = lo; i < hi; ++i) {
      const double dx = obs[i][0] - c[0], dy = obs[i][1] - c[1], dz = obs[i][2] - c[2];
      c[3] = std::max(c[3], std::sqrt(dx * dx + dy * dy + dz * dz) + obs[i][3]);
    }
    c[3] += kBoundMargin;
    cl.push_back(c);
    rg.push_back({lo, hi});
    return;
  }
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int i = lo; i < hi; ++i)
    for (int a = 0; a < 3; ++a) { mn[a] = std::min(mn[a], obs[i][a]); mx[a] = std::max(mx[a], obs[i][a]); }
  int ax = 0;
  for (int a = 1; a < 3; ++a) if (mx[a] - mn[a] > mx[ax] - mn[ax]) ax = a;
  const int mid = (lo + hi) / 2;
  std::nth_element(obs.begin() + lo, obs.begin() + mid, obs.begin() + hi,
                   [ax](const std::array<double, 4>& x, const std::array<double, 4>& y) { return x[ax] < y[ax]; });
  build_clusters(obs, lo, mid, cl, rg);
  build_clusters(obs, mid, hi, cl, rg);
}

// Link bounding spheres and the box around all obstacles (both inflated by kBoundMargin).
struct HBounds {
  double lbs[MAXJ][4];
  double lo[3], hi[3];
};

template <class T>
void fill_tp(TP<T>& t, const HScene& s, const std::vector<HT>& tref, const std::vector<double>& submass, double Mtot,
             const HBounds& hb) {
  std::memset(&t, 0, sizeof(TP<T>));
  for (size_t j = 0; j < s.joints.size() && j < MAXJ; ++j) {
    for (int k = 0; k < 9; ++k) t.jR[j][k] = T(s.joints[j].R[k]);
    for (int k = 0; k < 3; ++k) t.jp[j][k] = T(s.joints[j].p[k]);
    t.mass[j] = T(s.mass[j]);
    for (int k = 0; k < 3; ++k) t.mcom[j][k] = T(s.mass[j] * s.com[j][k]);
    t.submass[j] = T(submass[j]);
  }
  for (size_t f = 0; f < s.frames.size() && f < MAXF; ++f) {
    for (int k = 0; k < 9; ++k) t.fR[f][k] = T(s.frames[f].R[k]);
    for (int k = 0; k < 3; ++k) t.fp[f][k] = T(s.frames[f].p[k]);
  }
  for (size_t b = 0; b < s.blocks.size() && b < MAXB; ++b) {
    const HT& r = tref[b];
    for (int i = 0; i < 3; ++i) for (int k = 0; k < 3; ++k) t.refRt[b][3 * i + k] = T(r.R[3 * k + i]);
    for (int k = 0; k < 3; ++k) t.refp[b][k] = T(r.p[k]);
    for (int k = 0; k < 3; ++k) t.target[b][k] = T(s.blocks[b].target[k]);
    if (s.blocks[b].type == B_POSE && (s.blocks[b].aux & BF_BOUNDED))
      for (int c = 0; c < 6; ++c) {
        t.blo[b][c] = T(s.blocks[b].ext[c]);
        t.bhi[b][c] = T(s.blocks[b].ext[6 + c]);
      }
    if (s.blocks[b].type == B_HULL) {
      const int nv = s.blocks[b].aux;
      const double* V = s.blocks[b].ext;
      for (int i = 0; i < nv && i < MAXHV; ++i) {
        const double ax = V[2 * i], ay = V[2 * i + 1];
        const double ex = V[2 * ((i + 1) % nv)] - ax, ey = V[2 * ((i + 1) % nv) + 1] - ay;
        const double len = std::sqrt(ex * ex + ey * ey);
        t.hull_e[i][0] = T(ax); t.hull_e[i][1] = T(ay); t.hull_e[i][2] = T(ex); t.hull_e[i][3] = T(ey);
        // outward normal of a counter-clockwise polygon: the edge direction turned clockwise
        t.hull_n[i][0] = T(ey / len); t.hull_n[i][1] = T(-ex / len); t.hull_n[i][2] = T(1.0 / (len * len));
      }
    }
  }
  t.inv_total_mass = Mtot > 0 ? T(1.0 / Mtot) : T(0);
  for (int l = 0; l < MAXJ; ++l)
    for (int k = 0; k < 4; ++k) t.lbs[l][k] = float(hb.lbs[l][k]);
  for (int k = 0; k < 3; ++k) {
    t.obs_lo[k] = float(hb.lo[k]);
    t.obs_hi[k] = float(hb.hi[k]);
  }
  if (s.family == MC_FAMILY_LINEAR) {
    for (int r = 0; r < s.m; ++r) {
      for (int c = 0; c < s.d; ++c) t.A[r][c] = T(s.A[size_t(r) * s.d + c]);
      t.b[r] = T(s.b[r]);
    }
  }
}

// ------------------------------------------------------------------ utility kernels
__global__ void k_reset_u32(unsigned int* p, int n) {
  if (int(threadIdx.x) < n) p[threadIdx.x] = 0u;
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <class IO>
__global__ void k_zero1(IO* p) { *p = IO(0); }

__device__ __forceinline__ int find_geo(const int32_t* offs, int n_geo, int64_t i) {
  int lo = 0, hi = n_geo;  // offs[lo] <= i < offs[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offs[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

template <class IO>
__global__ void k_interpolate(int n_geo, const int32_t* offs, const IO* e, int64_t ld_e, int64_t total, IO* q,
                              int64_t ld, int d) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total || i >= int64_t(offs[n_geo])) return;
  const int g = find_geo(offs, n_geo, i);
  const int L = offs[g + 1] - offs[g];
  if (L <= 0) return;
  const double t = double(i - offs[g] + 1) / double(L + 1);
  for (int c = 0; c < d; ++c) {
    const double a = double(e[c * ld_e + 2 * g]), b = double(e[c * ld_e + 2 * g + 1]);
    q[c * ld + i] = IO(a + t * (b - a));
  }
}

// The geodesic holding configuration i, found by one wavefront: each round, the 64 lanes probe
// 64 evenly spaced offsets and a ballot narrows the range 64-fold (2 rounds for 4,096 geodesics,
// against 12 dependent loads of a binary search). Call with all 64 lanes of the wave active.
__device__ __forceinline__ int half_wave_find_geo(const int32_t* offs, int n_geo, int64_t i) {
  int lo = 0, hi = n_geo;  // offs[lo] <= i < offs[hi] (or hi = n_geo)
  const int lane = int(threadIdx.x & 31), half = int(threadIdx.x >> 5) & 1;
  while (hi - lo > 1) {  // uniform within each half-wave
    const int64_t span = hi - lo;
    const int probe = lo + int((span * lane) / 32);
    const bool le = lane == 0 || offs[probe] <= i;  // offs[probe] <= i (lane 0 probes lo)
    const uint32_t m = uint32_t(uint64_t(__ballot(le)) >> (32 * half));
    const int last = 31 - __builtin_clz(m);  // the highest probe still <= i
    const int nlo = lo + int((span * last) / 32);
    const int nhi = last == 31 ? hi : lo + int((span * (last + 1)) / 32);
    lo = nlo;
    hi = nhi > nlo ? nhi : nlo + 1;
  }
  return lo;
}

// The geodesics a workgroup's configurations [i0, i1] belong to: the first wavefront finds the
// first (lanes 0-31) and the last one (lanes 32-63) in 32-ary searches side by side, the workgroup
// stages the offsets between them in LDS (when they fit) and searches there.
constexpr int kGeoWindow = 1024;
constexpr int kMaxD = 36;  // largest configuration dimension of the compiled families

template <class IO>
__global__ void __launch_bounds__(256) k_path_grad(int64_t n, const IO* q, int64_t ld, const int32_t* offs, int n_geo,
                                                   IO* g, IO* loss, int d) {
  __shared__ int32_t s_offs[kGeoWindow];
  __shared__ int s_g[2];
  const int64_t i0 = int64_t(blockIdx.x) * blockDim.x;
  const int64_t i1 = (i0 + blockDim.x < n ? i0 + blockDim.x : n) - 1;
  const int64_t i = i0 + threadIdx.x;
  const bool act = i < n;
  // the configuration's own coordinates are requested first, so that their latency overlaps the
  // geodesic search
  IO x[kMaxD];
  for (int c = 0; c < kMaxD; ++c) x[c] = (act && c < d) ? q[int64_t(c) * ld + i] : IO(0);
  if (threadIdx.x < 64) {
    const int gx = half_wave_find_geo(offs, n_geo, threadIdx.x < 32 ? i0 : i1);
    if ((threadIdx.x & 31) == 0) s_g[threadIdx.x >> 5] = gx;
  }
  __syncthreads();
  const int g0 = s_g[0], w = s_g[1] - g0 + 2;  // offsets g0 .. g1 + 1
  const bool win = w <= kGeoWindow;
  if (win)
    for (int t = threadIdx.x; t < w; t += blockDim.x) s_offs[t] = offs[g0 + t];
  __syncthreads();
  int64_t lo_off = 0, hi_off = 0;  // the configuration's geodesic is [lo_off, hi_off)
  if (act) {
    if (win) {
      int lo = 0, hi = w - 1;  // s_offs[lo] <= i < s_offs[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_offs[mid] <= i) lo = mid; else hi = mid;
      }
      lo_off = s_offs[lo];
      hi_off = s_offs[lo + 1];
    } else {
      const int gi = find_geo(offs, n_geo, i);
      lo_off = offs[gi];
      hi_off = offs[gi + 1];
    }
  }
  // the searches clamp to the first and last geodesic: a configuration before geo_offsets[0] or
  // from geo_offsets[n_geo] on lies on none
  const bool inside = act && lo_off <= i && i < hi_off;
  const bool has_prev = inside && i > lo_off, has_next = inside && i + 1 < hi_off && i + 1 < n;
  // each coordinate is read once: the neighbours' come from the adjacent lanes, and only the
  // wave's first and last lanes read the configuration outside the wave
  const int lane = int(threadIdx.x & 63);
  IO xp[kMaxD], xn[kMaxD];
  for (int c = 0; c < kMaxD; ++c) {
    xp[c] = __shfl_up(x[c], 1u);
    xn[c] = __shfl_down(x[c], 1u);
  }
  if (lane == 0 && has_prev)
    for (int c = 0; c < kMaxD; ++c)
      if (c < d) xp[c] = q[int64_t(c) * ld + i - 1];
  if (lane == 63 && has_next)
    for (int c = 0; c < kMaxD; ++c)
      if (c < d) xn[c] = q[int64_t(c) * ld + i + 1];
  double seg = 0.0;
  if (act) {
    double np = 0.0, nn = 0.0;
    for (int c = 0; c < kMaxD; ++c) {
      const double tp = has_prev ? double(x[c]) - double(xp[c]) : 0.0;
      const double tn = has_next ? double(xn[c]) - double(x[c]) : 0.0;
      np += tp * tp;
      nn += tn * tn;
    }
    np = sqrt(np);
    nn = sqrt(nn);
    const double ip = 1.0 / fmax(np, 1e-12), in = 1.0 / fmax(nn, 1e-12);
    for (int c = 0; c < kMaxD; ++c) {
      if (c < d) {
        double gr = 0.0;
        if (has_prev) gr += (double(x[c]) - double(xp[c])) * ip;  // u_{i-1}
        if (has_next) gr -= (double(xn[c]) - double(x[c])) * in;  // -u_i
        g[int64_t(c) * ld + i] = IO(gr);
      }
    }
    if (has_next) seg = nn;
  }
  // wave reduction, then the workgroup's waves through LDS: one atomic per workgroup
  for (int off = 32; off > 0; off >>= 1) seg += __shfl_xor(seg, off);
  __shared__ double part[4];  // launched with 256 threads
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = seg;
  __syncthreads();
  if (loss && threadIdx.x == 0) {
    const double t = part[0] + part[1] + part[2] + part[3];
    if (t != 0.0) atomicAdd(loss, IO(t));
  }
}

__global__ void k_geo_ok(int n_geo, const int32_t* offs, int64_t n, const int8_t* status, const uint8_t* verdict, uint8_t* ok) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_geo) return;
  uint8_t r = 1;
  const int64_t lo = offs[g] < 0 ? 0 : offs[g];
  const int64_t hi = offs[g + 1] < n ? offs[g + 1] : n;
  for (int64_t i = lo; i < hi; ++i) {
    if (status[i] != ST_CONVERGED) r = 0;
    if (verdict && verdict[i] != V_FREE) r = 0;
  }
  ok[g] = r;
}


// ------------------------------------------------------------ ConstrainedExtend
// Alg. 2 ConstrainedExtend batched over independent extensions. Each extension keeps a chain of
// K = (n + 1) 2^Lmax + 1 points in the call's element type (every chain point is a start or a
// projected point of that type), stored position-major ([d][K][E]: coordinate k of position pos
// of extension e at (k K + pos) E + e, so threads of neighbouring extensions touch neighbouring
// addresses): level 0 fills positions k 2^Lmax, level l the odd multiples of 2^(Lmax - l).
// Particles are numbered i E + e. The projections run in project_batch; these kernels build the
// batches and take the decisions.
constexpr int kExtRunning = -1;
constexpr int kExtNone = 127;  // no failure recorded at this level

// The glue kernels below read every coordinate they need into registers first (a fixed trip
// count of kMaxD with guards, fully unrolled), so each thread waits for memory once.

// particles p_i = q_steer + eps_i v (one thread per particle, particle i of extension e at i E + e)
template <class T>
__global__ void __launch_bounds__(256) k_ext_particles(int64_t E, int n, int d, const T* qs, const T* qt, int64_t ld, const T* eps, double r,
                                T* part, int64_t ldp, double* dist, int8_t* result, int32_t* particle, int32_t* npts) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= E * n) return;
  const int64_t i = g / E, e = g - i * E;
  double a[kMaxD], v[kMaxD];
#pragma unroll
  for (int c = 0; c < kMaxD; ++c) {
    a[c] = c < d ? double(qs[c * ld + e]) : 0.0;
    v[c] = c < d ? double(qt[c * ld + e]) : 0.0;
  }
  const double ep = double(eps[e * n + i]);
  double L2 = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxD; ++c) {
    v[c] -= a[c];
    L2 += v[c] * v[c];
  }
  const double L = sqrt(L2);
  const double ds = L < r ? L : r;
  const double f = L > 0.0 ? (ds + ep) / L : 0.0;
#pragma unroll
  for (int c = 0; c < kMaxD; ++c)
    if (c < d) part[c * ldp + g] = T(a[c] + f * v[c]);
  if (i == 0) {
    dist[e] = ds;
    result[e] = L > 0.0 ? int8_t(kExtRunning) : int8_t(MC_EXT_ZERO);
    particle[e] = -1;
    npts[e] = 0;
  }
}

// earliest converged particle, its collision verdict and distance test; seeds the chain ends
template <class T>
__global__ void __launch_bounds__(256) k_ext_select(int64_t E, int n, int d, const T* qs, int64_t ld, const T* pout, int64_t ldp,
                             const int8_t* st, const int8_t* it, const uint8_t* vd, const double* dist, int8_t* result,
                             int32_t* particle, T* q_out, int64_t ld_out, T* chain, int64_t K, int64_t H) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E || result[e] != kExtRunning) return;
  int best = -1, best_it = 1 << 30;
  for (int i = 0; i < n; ++i) {
    const int64_t g = int64_t(i) * E + e;
    if (st[g] == ST_CONVERGED && int(it[g]) < best_it) {
      best = i;
      best_it = it[g];
    }
  }
  if (best < 0) {
    result[e] = MC_EXT_NO_PARTICLE;
    return;
  }
  particle[e] = best;
  const int64_t g = int64_t(best) * E + e;
  const int64_t cs = E * K, end = (int64_t(n) + 1) * H * E;
  T qa[kMaxD], qb[kMaxD];
#pragma unroll
  for (int c = 0; c < kMaxD; ++c) {
    qa[c] = c < d ? qs[c * ld + e] : T(0);
    qb[c] = c < d ? pout[c * ldp + g] : T(0);
  }
  double s2 = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxD; ++c) {
    if (c < d) {
      chain[c * cs + e] = qa[c];
      chain[c * cs + end + e] = qb[c];
      q_out[c * ld_out + e] = qb[c];
    }
    const double t = double(qb[c]) - double(qa[c]);
    s2 += t * t;
  }
  if (vd[g] != V_FREE) result[e] = MC_EXT_COLLISION;
  else if (sqrt(s2) > 2.0 * dist[e]) result[e] = MC_EXT_TOO_FAR;
}

// Level bookkeeping, one thread per extension: applies the previous level's failure code, ends
// extensions whose chain meets the resolution, and gives each extension that goes on a slot of
// the level's batch (wave-aggregated atomic).
__global__ void __launch_bounds__(256) k_ext_level(int64_t E, int n, int level, int lmax, double delta, int8_t* result, int32_t* npts,
                            int32_t* code, unsigned long long* maxgap, int32_t* slot_ext, unsigned int* count) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  bool alive = false;
  if (e < E && result[e] == kExtRunning) {
    if (level > 0) {
      if (code[e] != kExtNone) {
        result[e] = int8_t(code[e]);
      } else if (__longlong_as_double((long long)maxgap[e]) <= delta || level > lmax) {
        result[e] = MC_EXT_OK;
        npts[e] = int32_t((int64_t(n) + 1) << (level - 1)) + 1;
      } else {
        alive = true;
      }
    } else {
      alive = true;
    }
    if (level > lmax) alive = false;
    if (alive) {
      code[e] = kExtNone;
      maxgap[e] = 0ull;
    }
  }
  const uint64_t m = uint64_t(__ballot(alive));
  if (m == 0) return;
  const int lane = int(threadIdx.x & 63);
  const int leader = __builtin_ctzll(m);
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(count, (unsigned int)__builtin_popcountll(m));
  base = __shfl(base, leader);
  if (alive) slot_ext[base + __builtin_popcountll(m & ((1ull << lane) - 1ull))] = int32_t(e);
}

// Point g of a level's batch: new point j of the extension in slot s, numbered g = j alive + s
// (neighbouring threads: the same point of neighbouring extensions). Its chain position and the
// positions of its two neighbours.
struct ExtPoint {
  int64_t e, j, pos, lo, hi;
};
__device__ __forceinline__ ExtPoint ext_point(int64_t g, int64_t alive, int level, int64_t H, const int32_t* slot_ext) {
  ExtPoint p;
  p.j = g / alive;
  p.e = slot_ext[g - p.j * alive];
  if (level == 0) {
    p.pos = (p.j + 1) * H;
    p.lo = p.j * H;
    p.hi = (p.j + 2) * H;
  } else {
    const int64_t h = H >> level;
    p.pos = (2 * p.j + 1) * h;
    p.lo = 2 * p.j * h;
    p.hi = (2 * p.j + 2) * h;
  }
  return p;
}

// the level's new points: level 0 interpolates s + k/(n+1) (q_proj - s), later levels take the
// midpoint of every gap
template <class T>
__global__ void __launch_bounds__(256) k_ext_emit(int64_t total, int64_t alive, int n, int d, int level, int64_t E, const T* chain,
                           int64_t K, int64_t H, const int32_t* slot_ext, T* pts, int64_t ldx) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const ExtPoint p = ext_point(g, alive, level, H, slot_ext);
  const T* c = chain + p.e;
  const int64_t cs = E * K;
  // level 0: the chain's two ends and the chord fraction; later levels: the gap's two ends, halved
  const int64_t ia = level == 0 ? 0 : p.lo * E, ib = level == 0 ? (int64_t(n) + 1) * H * E : p.hi * E;
  const double t = level == 0 ? double(p.j + 1) / double(n + 1) : 0.5;
  T xa[kMaxD], xb[kMaxD];
#pragma unroll
  for (int k = 0; k < kMaxD; ++k) {
    xa[k] = k < d ? c[k * cs + ia] : T(0);
    xb[k] = k < d ? c[k * cs + ib] : T(0);
  }
#pragma unroll
  for (int k = 0; k < kMaxD; ++k) {
    const double a = double(xa[k]), b = double(xb[k]);
    if (k < d) pts[k * ldx + g] = T(level == 0 ? a + t * (b - a) : t * (a + b));
  }
}

// projected points into the chain, with their convergence and collision failures
template <class T>
__global__ void __launch_bounds__(256) k_ext_store(int64_t total, int64_t alive, int d, int level, int64_t E, T* chain, int64_t K,
                            int64_t H, const int32_t* slot_ext, const T* pout, int64_t ldx, const int8_t* st,
                            const uint8_t* vd, int32_t* code) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const ExtPoint p = ext_point(g, alive, level, H, slot_ext);
  const int64_t cs = E * K;
  T x[kMaxD];
#pragma unroll
  for (int k = 0; k < kMaxD; ++k) x[k] = k < d ? pout[k * ldx + g] : T(0);
#pragma unroll
  for (int k = 0; k < kMaxD; ++k)
    if (k < d) chain[k * cs + p.pos * E + p.e] = x[k];
  if (st[g] != ST_CONVERGED) atomicMin(code + p.e, int32_t(MC_EXT_INTERP_FAILED));
  else if (vd[g] != V_FREE) atomicMin(code + p.e, int32_t(MC_EXT_INTERP_COLLISION));
}

// the two gaps next to each new point against the level's bound r / (n 2^level); the longest
// gap of each extension (non-negative doubles order like their bit patterns)
template <class T>
__global__ void __launch_bounds__(256) k_ext_gaps(int64_t total, int64_t alive, int d, int level, int64_t E, const T* chain, int64_t K,
                           int64_t H, const int32_t* slot_ext, double bound, int32_t* code, unsigned long long* maxgap) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const ExtPoint p = ext_point(g, alive, level, H, slot_ext);
  const T* c = chain + p.e;
  const int64_t cs = E * K;
  T x[kMaxD], xl[kMaxD], xh[kMaxD];
#pragma unroll
  for (int k = 0; k < kMaxD; ++k) {
    x[k] = k < d ? c[k * cs + p.pos * E] : T(0);
    xl[k] = k < d ? c[k * cs + p.lo * E] : T(0);
    xh[k] = k < d ? c[k * cs + p.hi * E] : T(0);
  }
  double a2 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxD; ++k) {
    const double u = double(x[k]) - double(xl[k]), w = double(xh[k]) - double(x[k]);
    a2 += u * u;
    b2 += w * w;
  }
  const double gap = fmax(sqrt(a2), sqrt(b2));
  if (gap > bound) atomicMin(code + p.e, int32_t(MC_EXT_GAP));
  atomicMax(maxgap + p.e, (unsigned long long)__double_as_longlong(gap));
}

}  // namespace

struct mc_problem {
  int family = 0, d = 0, m = 0, device = 0, n_cu = 0;
  size_t max_lds_per_block = 0;
  DevProblem* dev = nullptr;
  float4* obs = nullptr;
  int n_obs = 0, n_sph = 0;
  unsigned int* counter = nullptr;  // [0] work-queue head, [1] projection FP64 queue, [2] VJP FP64 queue,
                                    // [3] exact-check queue
  unsigned long long* fallback = nullptr;
  // FP64 tail queues (FP32 mode), grown to the largest batch seen; calls on one handle must not
  // overlap (one stream at a time).
  mutable double* defer_q = nullptr;
  mutable int32_t* defer_ik = nullptr;
  mutable double* chk_q = nullptr;
  mutable int32_t* chk_idx = nullptr;
  mutable int64_t defer_cap = 0;
  mutable int32_t* vjp_idx = nullptr;
  mutable int64_t vjp_cap = 0;
  // resident workgroups per CU of the persistent kernel, by (FP64 mode, waves per block = 1, 2, 4);
  // queried once, so later calls (and calls under stream capture) make no runtime query
  mutable int occ[2][3] = {{0, 0, 0}, {0, 0, 0}};
  mutable int occ_wide = 0;  // resident 256-thread workgroups per CU of the two-wave launch
  // launch shape stored by mc_autotune_project, by (FP64 mode, cyclic mode); waves_per_block 0 = none
  mc_launch_shape tuned[2][2] = {{{0, 0, 0}, {0, 0, 0}}, {{0, 0, 0}, {0, 0, 0}}};
  // mc_set_check_lanes: lanes per configuration of the exact-check tail (0: by queue length)
  int32_t check_lanes = 0;
  // lanes per configuration of the exact-check tail on long queues, as mc_autotune_project chose
  // them (0: not tuned, kTailCheckLanesLong)
  int32_t check_long = 0;
  // mc_set_kernel_timing: events around the main projection launch [0, 1] and the VJP launch [2, 3]
  bool timing = false;
  hipEvent_t tev[4] = {nullptr, nullptr, nullptr, nullptr};
  mutable bool timed[2] = {false, false};
  // extend_batch workspace (particle and level batches, chains, per-extension state), grown to
  // the largest call
  mutable unsigned char* x_arena = nullptr;
  mutable size_t x_bytes = 0;
};

// Grow a tail queue to hold n entries (synchronises the device when it reallocates).
static hipError_t grow_defer(const mc_problem* p, int64_t n, int dmax) {
  if (n <= p->defer_cap) return hipSuccess;
  hipError_t e;
  for (void* b : {(void*)p->defer_q, (void*)p->defer_ik, (void*)p->chk_q, (void*)p->chk_idx})
    if (b && (e = hipFree(b)) != hipSuccess) return e;
  p->defer_q = nullptr;
  p->defer_ik = nullptr;
  p->chk_q = nullptr;
  p->chk_idx = nullptr;
  p->defer_cap = 0;
  if ((e = hipMalloc((void**)&p->defer_q, size_t(n) * size_t(dmax) * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&p->defer_ik, size_t(n) * 2 * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&p->chk_q, size_t(n) * size_t(dmax) * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&p->chk_idx, size_t(n) * sizeof(int32_t))) != hipSuccess) return e;
  p->defer_cap = n;
  return hipSuccess;
}
static hipError_t grow_vjp(const mc_problem* p, int64_t n) {
  if (n <= p->vjp_cap) return hipSuccess;
  hipError_t e;
  if (p->vjp_idx && (e = hipFree(p->vjp_idx)) != hipSuccess) return e;
  p->vjp_idx = nullptr;
  p->vjp_cap = 0;
  if ((e = hipMalloc((void**)&p->vjp_idx, size_t(n) * sizeof(int32_t))) != hipSuccess) return e;
  p->vjp_cap = n;
  return hipSuccess;
}

extern "C" {

const char* mc_last_error(void) { return g_err.c_str(); }

void mc_default_opts(mc_project_opts* o) {
  if (!o) return;
  o->dtype = MC_F32;
  o->tol = 1e-6;
  o->max_iter = 50;
  o->alpha = 1.0;
  o->lambda = 0.0;
  o->max_step = 0.0;
  o->fp64_cond_threshold = 1e6;
  o->check_collision = 1;
  o->variant = 0;
  o->waves_per_block = 0;
  o->blocks_per_cu = 0;
  o->mode = 0;
  o->lanes_per_config = 0;
  o->step_form = 0;
}

int32_t mc_problem_dof(const mc_problem* p) { return p ? p->d : -1; }
int32_t mc_problem_rows(const mc_problem* p) { return p ? p->m : -1; }
int32_t mc_problem_family(const mc_problem* p) { return p ? p->family : -1; }

void mc_problem_destroy(mc_problem* p) {
  if (!p) return;
  for (hipEvent_t& ev : p->tev)
    if (ev) (void)hipEventDestroy(ev);
  hipFree(p->dev);
  hipFree(p->obs);
  hipFree(p->counter);
  hipFree(p->fallback);
  hipFree(p->defer_q);
  hipFree(p->defer_ik);
  hipFree(p->chk_q);
  hipFree(p->chk_idx);
  hipFree(p->vjp_idx);
  hipFree(p->x_arena);
  delete p;
}

mc_status mc_problem_create(const void* blob, size_t nbytes, mc_problem** out) {
  g_err.clear();
  if (!blob || !out) return fail(MC_ERR_INVALID_ARG, "mc_problem_create: null argument");
  *out = nullptr;
  HScene s;
  std::string err;
  if (!parse_blob(blob, nbytes, s, err)) return fail(MC_ERR_INVALID_ARG, err);
  if (!validate_family(s, err)) return fail(MC_ERR_UNSUPPORTED, err);
  if (s.spheres.size() > size_t(MAXS)) return fail(MC_ERR_UNSUPPORTED, "too many robot spheres");

  // reference poses of blocks
  std::vector<HT> tref(s.blocks.size());
  std::vector<HT> Lref;
  if (!s.qref.empty() && !s.joints.empty()) Lref = host_fk(s, s.qref.data());
  auto frame_at = [&](int f) { return ht_mul(Lref[s.frames[f].link], ht_make(s.frames[f].R, s.frames[f].p)); };
  for (size_t b = 0; b < s.blocks.size(); ++b) {
    const auto& B = s.blocks[b];
    if (B.ref_from_qref && B.type == B_POSE) tref[b] = frame_at(B.fa);
    else if (B.ref_from_qref && B.type == B_REL) tref[b] = ht_mul(ht_inv(frame_at(B.fa)), frame_at(B.fb));
    else tref[b] = ht_make(B.R, B.p);
    if (B.ref_from_qref && B.type == B_DIST) {  // the rod length at q_ref
      const HT a = frame_at(B.fa), c = frame_at(B.fb);
      const double dx = c.p[0] - a.p[0], dy = c.p[1] - a.p[1], dz = c.p[2] - a.p[2];
      s.blocks[b].target[0] = std::sqrt(dx * dx + dy * dy + dz * dz);
    }
  }
  // subtree masses (joints are in depth-first preorder; parent < child)
  std::vector<double> submass(s.joints.size(), 0.0);
  double Mtot = 0.0;
  for (int j = int(s.joints.size()) - 1; j >= 0; --j) {
    submass[j] += s.mass[j];
    if (s.joints[j].parent >= 0) submass[s.joints[j].parent] += submass[j];
    Mtot += s.mass[j];
  }

  DevProblem* hp = new DevProblem;
  std::memset(hp, 0, sizeof(DevProblem));
  HBounds hb;
  std::memset(&hb, 0, sizeof hb);
  hp->c.dof = s.d;
  hp->c.rows = s.m;
  hp->c.lin_m = s.family == MC_FAMILY_LINEAR ? s.m : 0;
  hp->c.hull_nv = 0;
  for (const auto& B : s.blocks)
    if (B.type == B_HULL) hp->c.hull_nv = B.aux;
  CollConsts& K = hp->k;

  // robot spheres grouped by link, link bounding spheres
  std::vector<HSphere> sph = s.spheres;
  std::stable_sort(sph.begin(), sph.end(), [](const HSphere& a, const HSphere& b) { return a.link < b.link; });
  K.n_sph = int(sph.size());
  K.point_sph = make_float4(0.f, 0.f, 0.f, -1.f);
  int idx = 0;
  for (int l = 0; l <= MAXJ; ++l) K.sph_begin[l] = 0;
  std::vector<HSphere> linked;
  for (const auto& sp : sph) {
    if (sp.link < 0) K.point_sph = make_float4(float(sp.c[0]), float(sp.c[1]), float(sp.c[2]), float(sp.r));
    else linked.push_back(sp);
  }
  if (s.family == MC_FAMILY_SPHERE && sph.empty()) K.point_sph = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int l = 0; l < MAXJ; ++l) {
    K.sph_begin[l] = idx;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    const int first = idx;
    for (const auto& sp : linked) {
      if (sp.link != l) continue;
      K.sph[idx++] = make_float4(float(sp.c[0]), float(sp.c[1]), float(sp.c[2]), float(sp.r));
      for (int a = 0; a < 3; ++a) { mn[a] = std::min(mn[a], sp.c[a]); mx[a] = std::max(mx[a], sp.c[a]); }
    }
    if (idx > first) {
      const double c[3] = {0.5 * (mn[0] + mx[0]), 0.5 * (mn[1] + mx[1]), 0.5 * (mn[2] + mx[2])};
      double r = 0.0;
      for (const auto& sp : linked) {
        if (sp.link != l) continue;
        const double dx = sp.c[0] - c[0], dy = sp.c[1] - c[1], dz = sp.c[2] - c[2];
        r = std::max(r, std::sqrt(dx * dx + dy * dy + dz * dz) + sp.r);
      }
      K.link_bs[l] = make_float4(float(c[0]), float(c[1]), float(c[2]), float(r + kBoundMargin));
      hb.lbs[l][0] = c[0];
      hb.lbs[l][1] = c[1];
      hb.lbs[l][2] = c[2];
      hb.lbs[l][3] = r + kBoundMargin;
    } else {
      K.link_bs[l] = make_float4(0.f, 0.f, 0.f, -1.f);
      hb.lbs[l][3] = -1.0;
    }
  }
  for (int l = MAXJ; l < MAXJ + 4; ++l) K.sph_begin[l] = idx;

  // obstacle clusters
  std::vector<std::array<double, 4>> obs = s.obs;
  std::vector<std::array<double, 4>> cl;
  std::vector<std::array<int, 2>> rg;
  if (obs.size() > size_t(MAXO)) {
    delete hp;
    return fail(MC_ERR_UNSUPPORTED, "more than 2048 obstacle spheres");
  }
  if (!obs.empty()) build_clusters(obs, 0, int(obs.size()), cl, rg);
  if (cl.size() > size_t(MAXC)) {
    delete hp;
    return fail(MC_ERR_UNSUPPORTED, "too many obstacle clusters");
  }
  K.n_obs = int(obs.size());
  K.n_clus = int(cl.size());
  std::vector<float4> obs_f(obs.size());
  for (size_t i = 0; i < obs.size(); ++i) obs_f[i] = make_float4(float(obs[i][0]), float(obs[i][1]), float(obs[i][2]), float(obs[i][3]));
  // cluster boxes (bounding the obstacle spheres, inflated), then groups of up to kGroupSize
  // consecutive clusters (neighbours in the median-split order) with the union box
  std::vector<std::array<double, 6>> box(cl.size());
  for (size_t i = 0; i < cl.size(); ++i) {
    std::array<double, 6> b{1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
    for (int o = rg[i][0]; o < rg[i][1]; ++o)
      for (int a = 0; a < 3; ++a) {
        b[a] = std::min(b[a], obs[o][a] - obs[o][3]);
        b[3 + a] = std::max(b[3 + a], obs[o][a] + obs[o][3]);
      }
    for (int a = 0; a < 3; ++a) { b[a] -= kBoundMargin; b[3 + a] += kBoundMargin; }
    box[i] = b;
    K.clus_lo[i] = make_float4(float(b[0]), float(b[1]), float(b[2]), 0.f);
    K.clus_hi[i] = make_float4(float(b[3]), float(b[4]), float(b[5]), 0.f);
    K.clus_range[i] = make_int2(rg[i][0], rg[i][1]);
  }
  K.n_sup = 0;
  for (size_t c0 = 0; c0 < cl.size(); c0 += kGroupSize) {
    const size_t c1 = std::min(cl.size(), c0 + kGroupSize);
    std::array<double, 6> b{1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
    for (size_t c = c0; c < c1; ++c)
      for (int a = 0; a < 3; ++a) { b[a] = std::min(b[a], box[c][a]); b[3 + a] = std::max(b[3 + a], box[c][3 + a]); }
    K.sup_lo[K.n_sup] = make_float4(float(b[0]), float(b[1]), float(b[2]), 0.f);
    K.sup_hi[K.n_sup] = make_float4(float(b[3]), float(b[4]), float(b[5]), 0.f);
    K.sup_range[K.n_sup] = make_int2(int(c0), int(c1));
    ++K.n_sup;
  }

  // box around all obstacle spheres (an empty box, lo > hi, when there are none)
  for (int a = 0; a < 3; ++a) { hb.lo[a] = 1e30; hb.hi[a] = -1e30; }
  for (const auto& o : obs)
    for (int a = 0; a < 3; ++a) {
      hb.lo[a] = std::min(hb.lo[a], o[a] - o[3] - kBoundMargin);
      hb.hi[a] = std::max(hb.hi[a], o[a] + o[3] + kBoundMargin);
    }
  fill_tp<double>(hp->c.d, s, tref, submass, Mtot, hb);
  fill_tp<float>(hp->c.f, s, tref, submass, Mtot, hb);

  mc_problem* p = new mc_problem;
  p->family = s.family;
  p->d = s.d;
  p->m = s.m;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { delete p; delete hp; return hip_fail(e, "hipGetDevice"); }
  hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
  int lds = 0;
  hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
  p->max_lds_per_block = size_t(lds);
  auto alloc = [&](void** ptr, size_t bytes) -> hipError_t { return hipMalloc(ptr, bytes > 0 ? bytes : 16); };
  if ((e = alloc((void**)&p->dev, sizeof(DevProblem))) != hipSuccess ||
      (e = alloc((void**)&p->obs, obs_f.size() * sizeof(float4))) != hipSuccess ||
      (e = alloc((void**)&p->counter, 4 * sizeof(unsigned int))) != hipSuccess ||
      (e = alloc((void**)&p->fallback, sizeof(unsigned long long))) != hipSuccess) {
    mc_problem_destroy(p);
    delete hp;
    return hip_fail(e, "mc_problem_create: hipMalloc");
  }
  hp->obs = p->obs;
  hp->fallback_counter = p->fallback;
  p->n_obs = K.n_obs;
  p->n_sph = K.n_sph;
  const unsigned long long zero64 = 0;
  const unsigned int zero32[4] = {0, 0, 0, 0};
  if ((e = hipMemcpy(p->dev, hp, sizeof(DevProblem), hipMemcpyHostToDevice)) != hipSuccess ||
      (!obs_f.empty() && (e = hipMemcpy(p->obs, obs_f.data(), obs_f.size() * sizeof(float4), hipMemcpyHostToDevice)) != hipSuccess) ||

      (e = hipMemcpy(p->counter, zero32, sizeof zero32, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->fallback, &zero64, sizeof zero64, hipMemcpyHostToDevice)) != hipSuccess) {
    mc_problem_destroy(p);
    delete hp;
    return hip_fail(e, "mc_problem_create: hipMemcpy");
  }
  delete hp;
  *out = p;
  return MC_OK;
}

static bool lds_ok(const mc_problem* p, size_t bytes) { return bytes <= p->max_lds_per_block; }

static mc_status check_opts(const mc_problem* p, const mc_project_opts* o) {
  if (!o) return fail(MC_ERR_INVALID_ARG, "null opts");
  if (o->dtype != MC_F32 && o->dtype != MC_F64) return fail(MC_ERR_INVALID_ARG, "bad dtype");
  if (!(o->tol > 0) || !std::isfinite(o->tol)) return fail(MC_ERR_INVALID_ARG, "tol must be > 0");
  if (o->max_iter < 0 || o->max_iter > 127) return fail(MC_ERR_INVALID_ARG, "max_iter must be in 0..127");
  if (!(o->alpha > 0) || !std::isfinite(o->alpha)) return fail(MC_ERR_INVALID_ARG, "alpha must be > 0");
  if (!(o->lambda >= 0) || !std::isfinite(o->lambda)) return fail(MC_ERR_INVALID_ARG, "lambda must be >= 0");
  if (std::isnan(o->max_step)) return fail(MC_ERR_INVALID_ARG, "max_step is NaN");
  if (!(o->fp64_cond_threshold > 0)) return fail(MC_ERR_INVALID_ARG, "fp64_cond_threshold must be > 0");
  if (o->variant < 0 || o->variant > 2) return fail(MC_ERR_INVALID_ARG, "variant must be 0, 1 or 2");
  if (o->waves_per_block != 0 && o->waves_per_block != 1 && o->waves_per_block != 2 && o->waves_per_block != 4)
    return fail(MC_ERR_INVALID_ARG, "waves_per_block must be 0, 1, 2 or 4");
  if (o->blocks_per_cu < 0 || o->blocks_per_cu > 64) return fail(MC_ERR_INVALID_ARG, "blocks_per_cu must be 0..64");
  if (o->mode != 0 && o->mode != 1) return fail(MC_ERR_INVALID_ARG, "mode must be 0 (stacked) or 1 (cyclic)");
  if (o->mode == 1 && o->variant == 1) return fail(MC_ERR_UNSUPPORTED, "the cyclic mode runs in the fused variant only");
  if (o->lanes_per_config != 0 && o->lanes_per_config != 1)
    return fail(MC_ERR_UNSUPPORTED, "lanes_per_config must be 0 (auto) or 1");
  if (o->step_form != 0 && o->step_form != 1) return fail(MC_ERR_INVALID_ARG, "step_form must be 0 (inner) or 1 (outer)");
  if (o->step_form == 1) {
    if (!(o->lambda > 0)) return fail(MC_ERR_INVALID_ARG, "the outer step form needs lambda > 0");
    if (o->mode != 0) return fail(MC_ERR_UNSUPPORTED, "the outer step form runs in the stacked mode only");
    const FamilyOps* ops = ops_for(p->family, o->dtype == MC_F64);
    if (!ops || ops->dof_max > kOuterMaxD) return fail(MC_ERR_UNSUPPORTED, "the outer step form needs d <= 16");
  }
  return MC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free workspace
// project_batch_noalloc takes the queue counters and the FP64 and exact-check queues of its call
// from this file-scope array (one copy per device, kept until the process ends) instead of the
// problem's grown buffers. Its layout per call: 4 counters, then the FP64 queue (iterates, then
// index and step pairs) and the exact-check queue (configurations, then indices), sized for the
// call's n, each part 256-byte aligned.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices] = {};

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of the scratch layout for n configurations of dmax coordinates.
static size_t scratch_bytes(int64_t n, int dmax) {
  return align256(4 * sizeof(uint32_t)) + 2 * align256(size_t(n) * dmax * sizeof(double)) +
         align256(size_t(n) * 2 * sizeof(int32_t)) + align256(size_t(n) * sizeof(int32_t));
}

// The device address of `scratch` on the current device (looked up once per device, with that
// device current: the array's host-side name is not a device address).
static mc_status scratch_on_current_device(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "project_batch_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices) return fail(MC_ERR_UNSUPPORTED, "project_batch_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
      return hip_fail(e, "project_batch_noalloc: hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return MC_OK;
}

// Shared body of project_batch (noalloc = false: the problem's workspace, grown when a batch is
// larger than any before) and project_batch_noalloc (the device's scratch array).
static mc_status project_impl(const mc_problem* p, int64_t n, const void* q_in, int64_t ld_in, void* q_out, int64_t ld_out,
                              int8_t* status, int8_t* iters, void* resid, uint8_t* verdict, const int32_t* geo_offsets,
                              const int32_t* geo_offsets_host, int32_t n_geo, uint8_t* geo_ok,
                              const mc_project_opts* opts, void* stream, bool noalloc) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "project_batch: null problem");
  if (n < 0) return fail(MC_ERR_INVALID_ARG, "project_batch: n < 0");
  mc_status st = check_opts(p, opts);
  if (st != MC_OK) return st;
  if (n == 0) return MC_OK;
  if (!q_in || !q_out || !status || !iters || !resid) return fail(MC_ERR_INVALID_ARG, "project_batch: null array");
  if (ld_in < n || ld_out < n) return fail(MC_ERR_INVALID_ARG, "project_batch: ld < n");
  if (n > (int64_t(1) << 31) - 1) return fail(MC_ERR_INVALID_ARG, "project_batch: n too large");
  if (geo_ok && (!geo_offsets || n_geo <= 0)) return fail(MC_ERR_INVALID_ARG, "project_batch: geo_ok needs geo_offsets");
  int variant = opts->variant == 0 ? 2 : opts->variant;
  if (variant == 1) {
    if (!geo_offsets_host || n_geo <= 0) return fail(MC_ERR_INVALID_ARG, "project_batch: plain variant needs geo_offsets_host");
    if (geo_offsets_host[0] != 0 || geo_offsets_host[n_geo] != n) return fail(MC_ERR_INVALID_ARG, "project_batch: geo_offsets must span [0, n]");
    for (int g = 0; g < n_geo; ++g)
      if (geo_offsets_host[g + 1] < geo_offsets_host[g]) return fail(MC_ERR_INVALID_ARG, "project_batch: geo_offsets not monotone");
  }
  const FamilyOps* ops = ops_for(p->family, opts->dtype == MC_F64);
  if (!ops) return fail(MC_ERR_UNSUPPORTED, "project_batch: family without kernels");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* scr = nullptr;
  if (noalloc) {
    // the documented limit; the layout's alignment padding (< 1 KiB) fits below it
    const int64_t cap = int64_t((kScratchBytes - 1024) / (16 * size_t(ops->dof_max) + 12));
    if (n > cap || scratch_bytes(n, ops->dof_max) > kScratchBytes)
      return fail(MC_ERR_INVALID_ARG, "project_batch_noalloc: n = " + std::to_string(n) + " exceeds the scratch capacity of " +
                                          std::to_string(cap) + " configurations for this family");
    mc_status sst = scratch_on_current_device(&scr);
    if (sst != MC_OK) return sst;
  }
  unsigned int* counter = noalloc ? reinterpret_cast<unsigned int*>(scr) : p->counter;

  ProjArgs a;
  std::memset(&a, 0, sizeof a);
  a.P = p->dev;
  a.q_in = q_in;
  a.ld_in = ld_in;
  a.q_out = q_out;
  a.ld_out = ld_out;
  a.status = status;
  a.iters = iters;
  a.resid = resid;
  a.tol2 = opts->tol * opts->tol;
  a.alpha = opts->alpha;
  a.lambda = opts->lambda;
  a.max_step = opts->max_step;
  a.cond_thr = opts->fp64_cond_threshold;
  a.max_iter = opts->max_iter;
  a.check = opts->check_collision;
  a.outer = opts->step_form;
  a.counter = counter;
  a.n_sph = p->n_sph;
  a.n_obs = p->n_obs;
  a.chk_lanes = p->check_lanes;
  a.chk_long = p->check_long;
  hipError_t e;
  if (variant == 1) {
    a.verdict = verdict;
    if (p->timing && (e = hipEventRecord(p->tev[0], s)) != hipSuccess) return hip_fail(e, "project_batch: timing event");
    for (int g = 0; g < n_geo; ++g) {
      a.base = geo_offsets_host[g];
      a.n = geo_offsets_host[g + 1] - geo_offsets_host[g];
      if (a.n == 0) continue;
      if ((e = ops->project_plain(a, s)) != hipSuccess) return hip_fail(e, "project_batch: plain launch");
    }
    if (p->timing) {
      if ((e = hipEventRecord(p->tev[1], s)) != hipSuccess) return hip_fail(e, "project_batch: timing event");
      p->timed[0] = true;
    }
  } else {
    const bool cyc = opts->mode == 1;
    int wpb = opts->waves_per_block > 0 ? opts->waves_per_block : 1;
    int bpc = opts->blocks_per_cu;
    const mc_launch_shape& ts = p->tuned[ops->f64][cyc ? 1 : 0];
    const bool use_tuned = opts->variant == 0 && opts->waves_per_block == 0 && opts->blocks_per_cu == 0 &&
                           ts.waves_per_block > 0;
    if (use_tuned) {
      wpb = ts.waves_per_block;
      bpc = ts.blocks_per_cu;
    }
    while (wpb > 1 && (cyc ? 2 : 1) * ops->lds_bytes(64 * wpb) > p->max_lds_per_block) wpb >>= 1;
    const int block = 64 * wpb;
    const int bpc_req = bpc;  // 0: occupancy limit (and the two-wave build for large batches)
    if (bpc <= 0) {
      int& c = p->occ[ops->f64][wpb == 1 ? 0 : wpb == 2 ? 1 : 2];
      if (c <= 0) c = ops->persistent_blocks_per_cu(block);  // registers bound it, not LDS
      bpc = c;
    }
    int64_t grid = int64_t(p->n_cu) * bpc;
    // a batch beyond the lanes of the one-wave launch, with the launch shape left to the library:
    // the two-wave launch where the family has one
    const bool wide = !cyc && ops->project_persistent_wide != nullptr && bpc_req == 0 &&
                      n > grid * block && lds_ok(p, ops->lds_bytes(256));
    if (wide) {
      if (p->occ_wide <= 0) p->occ_wide = ops->persistent_wide_blocks_per_cu();
      grid = int64_t(p->n_cu) * p->occ_wide;
    }
    const int lblock = wide ? 256 : block;
    grid = std::min<int64_t>(grid, (n + lblock - 1) / lblock);
    a.base = 0;
    a.n = n;
    a.n_static = std::min<int64_t>(n, grid * lblock);
    const bool tail = ops->project_tail != nullptr;
    const bool ctail = verdict && opts->check_collision && ops->check_tail != nullptr;
    if (tail || ctail) {
      a.defer_count = counter + 1;
      a.chk_count = counter + 3;
      if (noalloc) {
        size_t off = align256(4 * sizeof(uint32_t));
        const size_t nq = align256(size_t(n) * ops->dof_max * sizeof(double));
        a.defer_q = reinterpret_cast<double*>(scr + off);
        off += nq;
        a.defer_ik = reinterpret_cast<int32_t*>(scr + off);
        off += align256(size_t(n) * 2 * sizeof(int32_t));
        a.chk_q = reinterpret_cast<double*>(scr + off);
        off += nq;
        a.chk_idx = reinterpret_cast<int32_t*>(scr + off);
        a.defer_cap = n;
      } else {
        if ((e = grow_defer(p, n, ops->dof_max)) != hipSuccess) return hip_fail(e, "project_batch: queue allocation");
        a.defer_ik = p->defer_ik;
        a.defer_q = p->defer_q;
        a.defer_cap = p->defer_cap;
        a.chk_idx = p->chk_idx;
        a.chk_q = p->chk_q;
      }
    }
    a.verdict = verdict;
    // counters cleared by a kernel (graph-capturable), never by a memset
    hipLaunchKernelGGL(k_reset_u32, dim3(1), dim3(64), 0, s, counter, 4);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "project_batch: reset");
    if (p->timing && (e = hipEventRecord(p->tev[0], s)) != hipSuccess) return hip_fail(e, "project_batch: timing event");
    if (wide) e = ops->project_persistent_wide(a, int(grid), s);
    else e = (cyc ? ops->project_persistent_cyclic : ops->project_persistent)(a, int(grid), block, s);
    if (e != hipSuccess) return hip_fail(e, "project_batch: persistent launch");
    if (p->timing) {
      if ((e = hipEventRecord(p->tev[1], s)) != hipSuccess) return hip_fail(e, "project_batch: timing event");
      p->timed[0] = true;
    }
    if (tail && (e = (cyc ? ops->project_tail_cyclic : ops->project_tail)(a, p->n_cu, s)) != hipSuccess)
      return hip_fail(e, "project_batch: FP64 tail launch");
    // 4 workgroups of 4 waves per CU: 4,096 work items per round (blocks without work leave at once)
    if (ctail && (e = ops->check_tail(a, kCheckTailBlocksPerCu * p->n_cu, s)) != hipSuccess) return hip_fail(e, "project_batch: check tail launch");
  }
  if (geo_ok) {
    hipLaunchKernelGGL(k_geo_ok, dim3((n_geo + 255) / 256), dim3(256), 0, s, n_geo, geo_offsets, n, status, verdict, geo_ok);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "project_batch: geo_ok");
  }
  return MC_OK;
}

extern "C" {

mc_status project_batch(const mc_problem* p, int64_t n, const void* q_in, int64_t ld_in, void* q_out, int64_t ld_out,
                        int8_t* status, int8_t* iters, void* resid, uint8_t* verdict, const int32_t* geo_offsets,
                        const int32_t* geo_offsets_host, int32_t n_geo, uint8_t* geo_ok, const mc_project_opts* opts,
                        void* stream) {
  return project_impl(p, n, q_in, ld_in, q_out, ld_out, status, iters, resid, verdict, geo_offsets, geo_offsets_host,
                      n_geo, geo_ok, opts, stream, false);
}

mc_status project_batch_noalloc(const mc_problem* p, int64_t n, const void* q_in, int64_t ld_in, void* q_out,
                                int64_t ld_out, int8_t* status, int8_t* iters, void* resid, uint8_t* verdict,
                                const int32_t* geo_offsets, const int32_t* geo_offsets_host, int32_t n_geo,
                                uint8_t* geo_ok, const mc_project_opts* opts, void* stream) {
  return project_impl(p, n, q_in, ld_in, q_out, ld_out, status, iters, resid, verdict, geo_offsets, geo_offsets_host,
                      n_geo, geo_ok, opts, stream, true);
}

mc_status check_batch(const mc_problem* p, int64_t n, const void* q, int64_t ld, mc_dtype dtype, uint8_t* verdict,
                      void* min_signed_dist, void* stream) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "check_batch: null problem");
  if (n < 0) return fail(MC_ERR_INVALID_ARG, "check_batch: n < 0");
  if (dtype != MC_F32 && dtype != MC_F64) return fail(MC_ERR_INVALID_ARG, "check_batch: bad dtype");
  if (n == 0) return MC_OK;
  if (!q || !verdict) return fail(MC_ERR_INVALID_ARG, "check_batch: null array");
  if (ld < n) return fail(MC_ERR_INVALID_ARG, "check_batch: ld < n");
  const FamilyOps* ops = ops_for(p->family, dtype == MC_F64);
  CheckArgs c;
  c.P = p->dev;
  c.n = n;
  c.q = q;
  c.ld = ld;
  c.status = nullptr;
  c.verdict = verdict;
  c.minsd = min_signed_dist;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (min_signed_dist || !ops->check_broad || !ops->check_tail) {
    if ((e = ops->check(c, min_signed_dist != nullptr, s)) != hipSuccess) return hip_fail(e, "check_batch: launch");
    return MC_OK;
  }
  // verdicts only: the broad phase of the fused projection, then the exact-check tail on the
  // configurations it queues (the problem's queue, grown to the largest batch seen)
  if ((e = grow_defer(p, n, ops->dof_max)) != hipSuccess) return hip_fail(e, "check_batch: queue allocation");
  ProjArgs a;
  std::memset(&a, 0, sizeof a);
  a.P = p->dev;
  a.verdict = verdict;
  a.chk_count = p->counter + 3;
  a.chk_idx = p->chk_idx;
  a.chk_q = p->chk_q;
  a.defer_cap = p->defer_cap;
  a.n_sph = p->n_sph;
  a.n_obs = p->n_obs;
  a.chk_lanes = p->check_lanes;
  a.chk_long = p->check_long;
  hipLaunchKernelGGL(k_reset_u32, dim3(1), dim3(64), 0, s, p->counter + 3, 1);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "check_batch: reset");
  if ((e = ops->check_broad(c, a.chk_count, a.chk_idx, a.chk_q, a.defer_cap, s)) != hipSuccess)
    return hip_fail(e, "check_batch: broad-phase launch");
  if ((e = ops->check_tail(a, kCheckTailBlocksPerCu * p->n_cu, s)) != hipSuccess) return hip_fail(e, "check_batch: exact-check launch");
  return MC_OK;
}

mc_status project_vjp(const mc_problem* p, int64_t n, const void* q_proj, int64_t ld, const int8_t* status,
                      const void* g_out, void* g_in, const mc_project_opts* opts, void* stream) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "project_vjp: null problem");
  if (n < 0) return fail(MC_ERR_INVALID_ARG, "project_vjp: n < 0");
  mc_status st = check_opts(p, opts);
  if (st != MC_OK) return st;
  if (n == 0) return MC_OK;
  if (!q_proj || !status || !g_out || !g_in) return fail(MC_ERR_INVALID_ARG, "project_vjp: null array");
  if (ld < n) return fail(MC_ERR_INVALID_ARG, "project_vjp: ld < n");
  const FamilyOps* ops = ops_for(p->family, opts->dtype == MC_F64);
  VjpArgs a;
  a.P = p->dev;
  a.n = n;
  a.q = q_proj;
  a.ld = ld;
  a.status = status;
  a.g = g_out;
  a.g_in = g_in;
  a.cond_thr = opts->fp64_cond_threshold;
  a.defer_count = nullptr;
  a.defer_idx = nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  const bool tail = ops->vjp_tail != nullptr;
  if (tail) {
    if ((e = grow_vjp(p, n)) != hipSuccess) return hip_fail(e, "project_vjp: FP64 queue allocation");
    a.defer_count = p->counter + 2;
    a.defer_idx = p->vjp_idx;
    hipLaunchKernelGGL(k_reset_u32, dim3(1), dim3(64), 0, s, p->counter + 2, 1);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "project_vjp: reset");
  }
  if (p->timing && (e = hipEventRecord(p->tev[2], s)) != hipSuccess) return hip_fail(e, "project_vjp: timing event");
  if ((e = ops->vjp(a, s)) != hipSuccess) return hip_fail(e, "project_vjp: launch");
  if (p->timing) {
    if ((e = hipEventRecord(p->tev[3], s)) != hipSuccess) return hip_fail(e, "project_vjp: timing event");
    p->timed[1] = true;
  }
  if (tail && (e = ops->vjp_tail(a, p->n_cu, s)) != hipSuccess) return hip_fail(e, "project_vjp: FP64 tail launch");
  return MC_OK;
}

mc_status project_vjp_exact(const mc_problem* p, int64_t n, const void* q_in, int64_t ld, const int8_t* status,
                            const int8_t* iters, const void* g_out, void* g_in, const mc_project_opts* opts,
                            void* stream) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "project_vjp_exact: null problem");
  if (n < 0) return fail(MC_ERR_INVALID_ARG, "project_vjp_exact: n < 0");
  mc_status st = check_opts(p, opts);
  if (st != MC_OK) return st;
  if (opts->mode != 0) return fail(MC_ERR_UNSUPPORTED, "project_vjp_exact: stacked mode only");
  if (n == 0) return MC_OK;
  if (!q_in || !status || !iters || !g_out || !g_in) return fail(MC_ERR_INVALID_ARG, "project_vjp_exact: null array");
  if (ld < n) return fail(MC_ERR_INVALID_ARG, "project_vjp_exact: ld < n");
  const FamilyOps* ops = ops_for(p->family, opts->dtype == MC_F64);
  VjpxArgs a;
  a.P = p->dev;
  a.n = n;
  a.q_in = q_in;
  a.ld = ld;
  a.status = status;
  a.iters = iters;
  a.g = g_out;
  a.g_in = g_in;
  a.alpha = opts->alpha;
  a.lambda = opts->lambda;
  a.h_rel = 1e-5;  // central-difference step of the Hessian-vector products, relative to max(1, |q|_inf)
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (p->timing && (e = hipEventRecord(p->tev[2], s)) != hipSuccess) return hip_fail(e, "project_vjp_exact: timing event");
  if ((e = ops->vjp_exact(a, s)) != hipSuccess) return hip_fail(e, "project_vjp_exact: launch");
  if (p->timing) {
    if ((e = hipEventRecord(p->tev[3], s)) != hipSuccess) return hip_fail(e, "project_vjp_exact: timing event");
    p->timed[1] = true;
  }
  return MC_OK;
}

mc_status interpolate_geodesics(const mc_problem* p, int32_t n_geo, const int32_t* geo_offsets, const void* endpoints,
                                int64_t ld_e, int64_t total, void* q_out, int64_t ld_out, mc_dtype dtype, void* stream) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "interpolate_geodesics: null problem");
  if (n_geo < 0 || total < 0) return fail(MC_ERR_INVALID_ARG, "interpolate_geodesics: negative size");
  if (n_geo == 0 || total == 0) return MC_OK;
  if (!geo_offsets || !endpoints || !q_out) return fail(MC_ERR_INVALID_ARG, "interpolate_geodesics: null array");
  if (ld_e < 2 * int64_t(n_geo)) return fail(MC_ERR_INVALID_ARG, "interpolate_geodesics: ld_e < 2 n_geo");
  if (dtype != MC_F32 && dtype != MC_F64) return fail(MC_ERR_INVALID_ARG, "interpolate_geodesics: bad dtype");
  if (total > (int64_t(1) << 31) - 1) return fail(MC_ERR_INVALID_ARG, "interpolate_geodesics: total too large");
  if (ld_out < total) return fail(MC_ERR_INVALID_ARG, "interpolate_geodesics: ld_out < total");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 g(unsigned((total + 255) / 256)), b(256);
  if (dtype == MC_F64)
    hipLaunchKernelGGL(k_interpolate<double>, g, b, 0, s, n_geo, geo_offsets, static_cast<const double*>(endpoints), ld_e,
                       total, static_cast<double*>(q_out), ld_out, p->d);
  else
    hipLaunchKernelGGL(k_interpolate<float>, g, b, 0, s, n_geo, geo_offsets, static_cast<const float*>(endpoints), ld_e,
                       total, static_cast<float*>(q_out), ld_out, p->d);
  hipError_t e;
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "interpolate_geodesics: launch");
  return MC_OK;
}

mc_status path_length_grad(const mc_problem* p, int64_t n, const void* q, int64_t ld, const int32_t* geo_offsets,
                           int32_t n_geo, void* g_out, void* loss, mc_dtype dtype, void* stream) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "path_length_grad: null problem");
  if (n < 0 || n_geo < 0) return fail(MC_ERR_INVALID_ARG, "path_length_grad: negative size");
  if (dtype != MC_F32 && dtype != MC_F64) return fail(MC_ERR_INVALID_ARG, "path_length_grad: bad dtype");
  if (n == 0) return MC_OK;
  if (!q || !geo_offsets || !g_out || n_geo == 0) return fail(MC_ERR_INVALID_ARG, "path_length_grad: null array");
  if (ld < n) return fail(MC_ERR_INVALID_ARG, "path_length_grad: ld < n");
  if (p->d > kMaxD) return fail(MC_ERR_UNSUPPORTED, "path_length_grad: dimension above 36");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  const dim3 g((n + 255) / 256), b(256);
  if (dtype == MC_F64) {
    if (loss) hipLaunchKernelGGL(k_zero1<double>, dim3(1), dim3(1), 0, s, static_cast<double*>(loss));
    hipLaunchKernelGGL(k_path_grad<double>, g, b, 0, s, n, static_cast<const double*>(q), ld, geo_offsets, n_geo,
                       static_cast<double*>(g_out), static_cast<double*>(loss), p->d);
  } else {
    if (loss) hipLaunchKernelGGL(k_zero1<float>, dim3(1), dim3(1), 0, s, static_cast<float*>(loss));
    hipLaunchKernelGGL(k_path_grad<float>, g, b, 0, s, n, static_cast<const float*>(q), ld, geo_offsets, n_geo,
                       static_cast<float*>(g_out), static_cast<float*>(loss), p->d);
  }
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "path_length_grad: launch");
  return MC_OK;
}

mc_status mc_eval_residual_jacobian(const mc_problem* p, int64_t n, const void* q, int64_t ld, mc_dtype dtype, void* F,
                                    void* J, void* stream) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "mc_eval_residual_jacobian: null problem");
  if (n < 0) return fail(MC_ERR_INVALID_ARG, "mc_eval_residual_jacobian: n < 0");
  if (dtype != MC_F32 && dtype != MC_F64) return fail(MC_ERR_INVALID_ARG, "mc_eval_residual_jacobian: bad dtype");
  if (n == 0) return MC_OK;
  if (!q || !F || !J) return fail(MC_ERR_INVALID_ARG, "mc_eval_residual_jacobian: null array");
  if (ld < n) return fail(MC_ERR_INVALID_ARG, "mc_eval_residual_jacobian: ld < n");
  const FamilyOps* ops = ops_for(p->family, dtype == MC_F64);
  hipError_t e = ops->eval_fj(p->dev, n, q, ld, F, J, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "mc_eval_residual_jacobian: launch");
  return MC_OK;
}

}  // extern "C"

// extend_batch workspace: every buffer 256-byte aligned inside one arena
struct ExtWs {
  double *pin, *pout, *chain, *rs, *dist;
  int8_t *st, *it;
  uint8_t* vd;
  int32_t *code, *slot_ext;
  unsigned long long* maxgap;
  unsigned int* count;
};
static size_t ext_layout(int64_t E, int64_t EK, int d, unsigned char* base, ExtWs* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* ptr = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return ptr;
  };
  unsigned char* pin = take(size_t(d) * EK * 8);
  unsigned char* pout = take(size_t(d) * EK * 8);
  unsigned char* chain = take(size_t(d) * EK * 8);
  unsigned char* rs = take(size_t(EK) * 8);
  unsigned char* dist = take(size_t(E) * 8);
  unsigned char* st = take(size_t(EK));
  unsigned char* it = take(size_t(EK));
  unsigned char* vd = take(size_t(EK));
  unsigned char* code = take(size_t(E) * 4);
  unsigned char* slot = take(size_t(E) * 4);
  unsigned char* mg = take(size_t(E) * 8);
  unsigned char* cnt = take(4);
  if (w) {
    w->pin = reinterpret_cast<double*>(pin);
    w->pout = reinterpret_cast<double*>(pout);
    w->chain = reinterpret_cast<double*>(chain);
    w->rs = reinterpret_cast<double*>(rs);
    w->dist = reinterpret_cast<double*>(dist);
    w->st = reinterpret_cast<int8_t*>(st);
    w->it = reinterpret_cast<int8_t*>(it);
    w->vd = reinterpret_cast<uint8_t*>(vd);
    w->code = reinterpret_cast<int32_t*>(code);
    w->slot_ext = reinterpret_cast<int32_t*>(slot);
    w->maxgap = reinterpret_cast<unsigned long long*>(mg);
    w->count = reinterpret_cast<unsigned int*>(cnt);
  }
  return off;
}

template <class T>
static mc_status extend_impl(const mc_problem* p, int64_t E, const T* qs, const T* qt, int64_t ld, const T* eps,
                             const mc_extend_opts* xo, const mc_project_opts* opts, T* q_out, int64_t ld_out,
                             int8_t* result, int32_t* particle, int32_t* npts, int lmax, hipStream_t s) {
  const int n = xo->n, d = p->d;
  const int64_t H = int64_t(1) << lmax, K = (int64_t(n) + 1) * H + 1, EK = E * K;
  const size_t need = ext_layout(E, EK, d, nullptr, nullptr);
  hipError_t e;
  if (need > p->x_bytes) {
    if (p->x_arena && (e = hipFree(p->x_arena)) != hipSuccess) return hip_fail(e, "extend_batch: free workspace");
    p->x_arena = nullptr;
    p->x_bytes = 0;
    if ((e = hipMalloc((void**)&p->x_arena, need)) != hipSuccess) return hip_fail(e, "extend_batch: workspace");
    p->x_bytes = need;
  }
  ExtWs w;
  ext_layout(E, EK, d, p->x_arena, &w);
  T* pin = reinterpret_cast<T*>(w.pin);
  T* pout = reinterpret_cast<T*>(w.pout);
  T* chain = reinterpret_cast<T*>(w.chain);
  mc_project_opts o = *opts;
  o.check_collision = 1;
  o.variant = 2;
  const int64_t np = E * n;
  hipLaunchKernelGGL(k_ext_particles<T>, dim3((np + 255) / 256), dim3(256), 0, s, E, n, d, qs, qt, ld, eps, xo->r,
                     pin, EK, w.dist, result, particle, npts);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "extend_batch: particles");
  mc_status st = project_batch(p, np, pin, EK, pout, EK, w.st, w.it, w.rs, w.vd, nullptr, nullptr, 0, nullptr, &o, s);
  if (st != MC_OK) return st;
  hipLaunchKernelGGL(k_ext_select<T>, dim3((E + 255) / 256), dim3(256), 0, s, E, n, d, qs, ld, pout, EK, w.st, w.it,
                     w.vd, w.dist, result, particle, q_out, ld_out, chain, K, H);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "extend_batch: select");
  for (int level = 0; level <= lmax + 1; ++level) {
    hipLaunchKernelGGL(k_reset_u32, dim3(1), dim3(64), 0, s, w.count, 1);
    hipLaunchKernelGGL(k_ext_level, dim3((E + 255) / 256), dim3(256), 0, s, E, n, level, lmax, xo->delta, result, npts,
                       w.code, w.maxgap, w.slot_ext, w.count);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "extend_batch: level");
    if (level > lmax) break;
    unsigned int alive = 0;
    if ((e = hipMemcpyAsync(&alive, w.count, sizeof alive, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(e, "extend_batch: read level size");
    if (alive == 0) break;
    const int64_t per = level == 0 ? int64_t(n) : (int64_t(n) + 1) << (level - 1);
    const int64_t total = int64_t(alive) * per;
    const dim3 g((total + 255) / 256), b(256);
    hipLaunchKernelGGL(k_ext_emit<T>, g, b, 0, s, total, int64_t(alive), n, d, level, E, chain, K, H, w.slot_ext,
                       pin, EK);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "extend_batch: emit");
    st = project_batch(p, total, pin, EK, pout, EK, w.st, w.it, w.rs, w.vd, nullptr, nullptr, 0, nullptr, &o, s);
    if (st != MC_OK) return st;
    hipLaunchKernelGGL(k_ext_store<T>, g, b, 0, s, total, int64_t(alive), d, level, E, chain, K, H, w.slot_ext, pout,
                       EK, w.st, w.vd, w.code);
    const double bound = xo->r / (double(n) * double(int64_t(1) << level));
    hipLaunchKernelGGL(k_ext_gaps<T>, g, b, 0, s, total, int64_t(alive), d, level, E, chain, K, H, w.slot_ext, bound,
                       w.code, w.maxgap);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "extend_batch: validate");
  }
  return MC_OK;
}

extern "C" {

mc_status extend_batch(const mc_problem* p, int64_t E, const void* q_start, const void* q_target, int64_t ld,
                       const void* eps, const mc_extend_opts* xo, const mc_project_opts* opts, void* q_out,
                       int64_t ld_out, int8_t* result, int32_t* particle, int32_t* n_points, void* stream) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "extend_batch: null problem");
  if (E < 0) return fail(MC_ERR_INVALID_ARG, "extend_batch: E < 0");
  mc_status st = check_opts(p, opts);
  if (st != MC_OK) return st;
  if (!xo) return fail(MC_ERR_INVALID_ARG, "extend_batch: null extend options");
  if (!(xo->r > 0) || !std::isfinite(xo->r)) return fail(MC_ERR_INVALID_ARG, "extend_batch: r must be > 0");
  if (!(xo->delta > 0) || !std::isfinite(xo->delta)) return fail(MC_ERR_INVALID_ARG, "extend_batch: delta must be > 0");
  if (xo->n < 1 || xo->n > 64) return fail(MC_ERR_INVALID_ARG, "extend_batch: n must be in 1..64");
  if (p->d > kMaxD) return fail(MC_ERR_UNSUPPORTED, "extend_batch: configuration dimension above 36");
  int lmax = 0;
  while (xo->r / (double(xo->n) * double(int64_t(1) << lmax)) > xo->delta) {
    if (++lmax > 12) return fail(MC_ERR_INVALID_ARG, "extend_batch: r / (n delta) needs more than 12 levels");
  }
  if ((int64_t(xo->n) + 1) << lmax > 65535) return fail(MC_ERR_INVALID_ARG, "extend_batch: chain longer than 65536");
  if (E == 0) return MC_OK;
  if (!q_start || !q_target || !eps || !q_out || !result || !particle || !n_points)
    return fail(MC_ERR_INVALID_ARG, "extend_batch: null array");
  if (ld < E || ld_out < E) return fail(MC_ERR_INVALID_ARG, "extend_batch: ld < E");
  const int64_t K = ((int64_t(xo->n) + 1) << lmax) + 1;
  if (E * K > (int64_t(1) << 31) - 1) return fail(MC_ERR_INVALID_ARG, "extend_batch: E times the chain length too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (opts->dtype == MC_F64)
    return extend_impl<double>(p, E, static_cast<const double*>(q_start), static_cast<const double*>(q_target), ld,
                               static_cast<const double*>(eps), xo, opts, static_cast<double*>(q_out), ld_out, result,
                               particle, n_points, lmax, s);
  return extend_impl<float>(p, E, static_cast<const float*>(q_start), static_cast<const float*>(q_target), ld,
                            static_cast<const float*>(eps), xo, opts, static_cast<float*>(q_out), ld_out, result,
                            particle, n_points, lmax, s);
}

mc_status mc_eval_condition(const mc_problem* p, int64_t n, const void* q, int64_t ld, mc_dtype dtype, double lambda,
                            void* kappa, void* stream) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "mc_eval_condition: null problem");
  if (n < 0) return fail(MC_ERR_INVALID_ARG, "mc_eval_condition: n < 0");
  if (dtype != MC_F32 && dtype != MC_F64) return fail(MC_ERR_INVALID_ARG, "mc_eval_condition: bad dtype");
  if (!(lambda >= 0) || !std::isfinite(lambda)) return fail(MC_ERR_INVALID_ARG, "mc_eval_condition: lambda must be >= 0");
  if (n == 0) return MC_OK;
  if (!q || !kappa) return fail(MC_ERR_INVALID_ARG, "mc_eval_condition: null array");
  if (ld < n) return fail(MC_ERR_INVALID_ARG, "mc_eval_condition: ld < n");
  const FamilyOps* ops = ops_for(p->family, dtype == MC_F64);
  hipError_t e = ops->eval_cond(p->dev, n, q, ld, lambda, kappa, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "mc_eval_condition: launch");
  return MC_OK;
}

mc_status mc_set_check_lanes(mc_problem* p, int32_t lanes) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "mc_set_check_lanes: null problem");
  if (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16 && lanes != 64)
    return fail(MC_ERR_INVALID_ARG, "mc_set_check_lanes: lanes must be 0, 1, 2, 4, 8, 16 or 64");
  p->check_lanes = lanes;
  return MC_OK;
}

mc_status mc_set_kernel_timing(mc_problem* p, int32_t on) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "mc_set_kernel_timing: null problem");
  if (on) {
    for (hipEvent_t& ev : p->tev) {
      if (ev) continue;
      hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return hip_fail(e, "mc_set_kernel_timing: event");
    }
  }
  p->timing = on != 0;
  p->timed[0] = p->timed[1] = false;
  return MC_OK;
}

mc_status mc_last_kernel_ms(const mc_problem* p, int32_t which, float* ms) {
  g_err.clear();
  if (!p || !ms) return fail(MC_ERR_INVALID_ARG, "mc_last_kernel_ms: null argument");
  if (which != 0 && which != 1) return fail(MC_ERR_INVALID_ARG, "mc_last_kernel_ms: which must be 0 or 1");
  if (!p->timed[which]) return fail(MC_ERR_INVALID_ARG, "mc_last_kernel_ms: no timed call of this kind");
  hipError_t e = hipEventSynchronize(p->tev[2 * which + 1]);
  if (e != hipSuccess) return hip_fail(e, "mc_last_kernel_ms: sync");
  if ((e = hipEventElapsedTime(ms, p->tev[2 * which], p->tev[2 * which + 1])) != hipSuccess)
    return hip_fail(e, "mc_last_kernel_ms: elapsed");
  return MC_OK;
}

mc_status mc_queue_counts(const mc_problem* p, uint32_t counts[4]) {
  g_err.clear();
  if (!p || !counts) return fail(MC_ERR_INVALID_ARG, "mc_queue_counts: null argument");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "mc_queue_counts: sync");
  if ((e = hipMemcpy(counts, p->counter, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "mc_queue_counts: read");
  return MC_OK;
}

}  // extern "C"

// Candidate launch shapes of the autotuner (waves per workgroup, workgroups per CU, lanes per
// configuration).
static const mc_launch_shape kTuneCandidates[] = {{1, 0, 1}, {2, 0, 1}, {4, 0, 1}, {1, 1, 1},
                                                  {1, 2, 1}, {2, 1, 1}, {4, 1, 1}};
constexpr int kNumTuneCandidates = int(sizeof(kTuneCandidates) / sizeof(kTuneCandidates[0]));

// Device outputs of one projection of the autotuner (one allocation).
struct TuneOut {
  unsigned char* base = nullptr;
  void *q = nullptr, *resid = nullptr;
  int8_t *status = nullptr, *iters = nullptr;
  uint8_t* verdict = nullptr;
  size_t bytes = 0;
  hipError_t alloc(int64_t n, int d, size_t elem) {
    const size_t nq = size_t(n) * d * elem, nr = size_t(n) * elem;
    bytes = nq + nr + 3 * size_t(n);
    hipError_t e = hipMalloc((void**)&base, bytes);
    if (e != hipSuccess) return e;
    q = base;
    resid = base + nq;
    status = reinterpret_cast<int8_t*>(base + nq + nr);
    iters = status + n;
    verdict = reinterpret_cast<uint8_t*>(iters + n);
    return hipSuccess;
  }
  ~TuneOut() {
    if (base) (void)hipFree(base);
  }
};

extern "C" {

int32_t mc_autotune_candidates(mc_launch_shape* shapes) {
  if (shapes)
    for (int c = 0; c < kNumTuneCandidates; ++c) shapes[c] = kTuneCandidates[c];
  return kNumTuneCandidates;
}

mc_status mc_autotune_project(mc_problem* p, int64_t n, const void* q_in, int64_t ld_in, const mc_project_opts* opts,
                              int32_t reps, void* stream, mc_launch_shape* best, float* ms) {
  g_err.clear();
  if (!p) return fail(MC_ERR_INVALID_ARG, "mc_autotune_project: null problem");
  mc_status st = check_opts(p, opts);
  if (st != MC_OK) return st;
  if (n <= 0 || !q_in) return fail(MC_ERR_INVALID_ARG, "mc_autotune_project: empty batch");
  if (ld_in < n) return fail(MC_ERR_INVALID_ARG, "mc_autotune_project: ld < n");
  if (reps < 1 || reps > 1000) return fail(MC_ERR_INVALID_ARG, "mc_autotune_project: reps must be in 1..1000");
  if (opts->variant == 1) return fail(MC_ERR_INVALID_ARG, "mc_autotune_project: tunes the fused variant");
  const size_t elem = opts->dtype == MC_F64 ? 8 : 4;
  hipStream_t s = static_cast<hipStream_t>(stream);
  TuneOut ref, cand;
  hipError_t e;
  if ((e = ref.alloc(n, p->d, elem)) != hipSuccess || (e = cand.alloc(n, p->d, elem)) != hipSuccess)
    return hip_fail(e, "mc_autotune_project: output buffers");
  std::vector<unsigned char> h_ref(ref.bytes), h_cand(cand.bytes);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e, "mc_autotune_project: events");
  }
  int best_c = -1;
  float best_ms = 0.f;
  mc_status rc = MC_OK;
  for (int c = 0; c < kNumTuneCandidates && rc == MC_OK; ++c) {
    mc_project_opts o = *opts;
    o.variant = 2;
    o.waves_per_block = kTuneCandidates[c].waves_per_block;
    o.blocks_per_cu = kTuneCandidates[c].blocks_per_cu;
    o.lanes_per_config = kTuneCandidates[c].lanes_per_config;
    TuneOut& out = c == 0 ? ref : cand;
    auto call = [&]() {
      return project_batch(p, n, q_in, ld_in, out.q, n, out.status, out.iters, out.resid,
                           o.check_collision ? out.verdict : nullptr, nullptr, nullptr, 0, nullptr, &o, stream);
    };
    if ((rc = call()) != MC_OK) break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(e, "mc_autotune_project: run"); break; }
    // every candidate must reproduce the first one bit for bit (the verdict bytes only when checked)
    const size_t cmp = o.check_collision ? out.bytes : out.bytes - size_t(n);
    if ((e = hipMemcpy(c == 0 ? h_ref.data() : h_cand.data(), out.base, cmp, hipMemcpyDeviceToHost)) != hipSuccess) {
      rc = hip_fail(e, "mc_autotune_project: read outputs");
      break;
    }
    if (c > 0 && std::memcmp(h_ref.data(), h_cand.data(), cmp) != 0) {
      rc = fail(MC_ERR_HIP, "mc_autotune_project: launch shape " + std::to_string(o.waves_per_block) + "x" +
                                std::to_string(o.blocks_per_cu) + " changed the results");
      break;
    }
    if ((e = hipEventRecord(e0, s)) != hipSuccess) { rc = hip_fail(e, "mc_autotune_project: event"); break; }
    for (int r = 0; r < reps && rc == MC_OK; ++r) rc = call();
    if (rc != MC_OK) break;
    float t = 0.f;
    if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
        (e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) {
      rc = hip_fail(e, "mc_autotune_project: timing");
      break;
    }
    t /= float(reps);
    if (ms) ms[c] = t;
    if (best_c < 0 || t < best_ms) {
      best_c = c;
      best_ms = t;
    }
  }
  // second stage, where the batch's exact-check queue is long (more entries than the tail's
  // wave-per-configuration path takes): the lane groups of that queue, in the best shape (groups of 1
  // and 2 only for the families that have them; the kernel rounds them up to 4 where the scene's
  // staged spheres leave no LDS room for them)
  mc_launch_shape chosen = kTuneCandidates[best_c >= 0 ? best_c : 0];
  unsigned queued = 0;
  if (rc == MC_OK && opts->check_collision &&
      (e = hipMemcpy(&queued, p->counter + 3, sizeof queued, hipMemcpyDeviceToHost)) != hipSuccess)
    rc = hip_fail(e, "mc_autotune_project: read the check queue length");
  if (rc == MC_OK && opts->check_collision && int64_t(queued) > int64_t(4) * kCheckTailBlocksPerCu * p->n_cu) {
    const int32_t saved = p->check_long;
    int32_t best_l = 0;
    float best_l_ms = 0.f;
    for (int32_t L : {1, 2, 4, 8, 16}) {
      if (L < 4 && p->d > kTailCheckLowLanesMaxD) continue;  // such families run groups of at least 4
      mc_project_opts o = *opts;
      o.variant = 2;
      o.waves_per_block = chosen.waves_per_block;
      o.blocks_per_cu = chosen.blocks_per_cu;
      o.lanes_per_config = chosen.lanes_per_config;
      p->check_long = L;
      auto call = [&]() {
        return project_batch(p, n, q_in, ld_in, cand.q, n, cand.status, cand.iters, cand.resid, cand.verdict, nullptr,
                             nullptr, 0, nullptr, &o, stream);
      };
      if ((rc = call()) != MC_OK) break;
      if ((e = hipMemcpy(h_cand.data(), cand.base, cand.bytes, hipMemcpyDeviceToHost)) != hipSuccess) {
        rc = hip_fail(e, "mc_autotune_project: read outputs");
        break;
      }
      if (std::memcmp(h_ref.data(), h_cand.data(), cand.bytes) != 0) {
        rc = fail(MC_ERR_HIP, "mc_autotune_project: exact-check lane groups of " + std::to_string(L) + " changed the results");
        break;
      }
      if ((e = hipEventRecord(e0, s)) != hipSuccess) { rc = hip_fail(e, "mc_autotune_project: event"); break; }
      for (int r = 0; r < reps && rc == MC_OK; ++r) rc = call();
      if (rc != MC_OK) break;
      float t = 0.f;
      if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
          (e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) {
        rc = hip_fail(e, "mc_autotune_project: timing");
        break;
      }
      t /= float(reps);
      if (best_l == 0 || t < best_l_ms) {
        best_l = L;
        best_l_ms = t;
      }
    }
    p->check_long = rc == MC_OK ? best_l : saved;
    chosen.check_lanes = best_l;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != MC_OK) return rc;
  p->tuned[opts->dtype == MC_F64 ? 1 : 0][opts->mode == 1 ? 1 : 0] = chosen;
  if (best) *best = chosen;
  return MC_OK;
}

mc_status mc_tuned_shape(const mc_problem* p, mc_dtype dtype, int32_t mode, mc_launch_shape* out) {
  g_err.clear();
  if (!p || !out) return fail(MC_ERR_INVALID_ARG, "mc_tuned_shape: null argument");
  if ((dtype != MC_F32 && dtype != MC_F64) || (mode != 0 && mode != 1)) return fail(MC_ERR_INVALID_ARG, "mc_tuned_shape: bad key");
  const mc_launch_shape& t = p->tuned[dtype == MC_F64 ? 1 : 0][mode];
  if (t.waves_per_block <= 0) return fail(MC_ERR_INVALID_ARG, "mc_tuned_shape: no shape stored for this key");
  *out = t;
  return MC_OK;
}

mc_status mc_fallback_count(const mc_problem* p, int reset, uint64_t* count) {
  g_err.clear();
  if (!p || !count) return fail(MC_ERR_INVALID_ARG, "mc_fallback_count: null argument");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "mc_fallback_count: sync");
  unsigned long long v = 0;
  if ((e = hipMemcpy(&v, p->fallback, sizeof v, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "mc_fallback_count: read");
  *count = v;
  if (reset) {
    const unsigned long long z = 0;
    if ((e = hipMemcpy(p->fallback, &z, sizeof z, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "mc_fallback_count: reset");
  }
  return MC_OK;
}

}  // extern "C"
