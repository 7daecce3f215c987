// Host side of the transport library: problem setup, the angular multigrid
// V-cycle (Fig. lmg), restarted GMRES and the adjoint gradient, behind the
// C ABI of tr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/tr.h"
#include "angular_setup.h"
#include "internal.h"

using tr::Grid;
using tr::OrdInfo;
using tr::Planes;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

struct HipError {
  hipError_t e;
  std::string where;
};

#define HIPCHK(call)                                                      \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) throw HipError{e_, #call};                      \
  } while (0)

struct ArgError {
  std::string msg;
};

// Psi = (3 I + J) / 6 and its inverse 2 I - J / 3 (identical on every patch).
const double kPsi[3][3] = {{4.0 / 6, 1.0 / 6, 1.0 / 6}, {1.0 / 6, 4.0 / 6, 1.0 / 6}, {1.0 / 6, 1.0 / 6, 4.0 / 6}};
const double kPsiInv[3][3] = {{5.0 / 3, -1.0 / 3, -1.0 / 3}, {-1.0 / 3, 5.0 / 3, -1.0 / 3}, {-1.0 / 3, -1.0 / 3, 5.0 / 3}};

void mat3_mul(const double *a, const double *b, double *c) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += a[i * 3 + k] * b[k * 3 + j];
      t[i * 3 + j] = s;
    }
  std::memcpy(c, t, sizeof t);
}

struct DevLevel {
  int P = 0, A = 0, order = 0;
  // forward sweep inputs (f and the post-smoothing right-hand side) are
  // kept in plane layout (see tr::SweepArgs::plane_in), per precision of
  // the V-cycle
  bool pin64 = false, pin32 = false;
  OrdInfo *ord = nullptr;
  double *w = nullptr, *winv = nullptr, *ipsi = nullptr;
  double *St64 = nullptr;      // canonical S~ (order of this level), A x A
  float *St32 = nullptr;
  double *G64 = nullptr, *Gt64 = nullptr;  // ordinate-form scatter and transpose
  float *G32 = nullptr, *Gt32 = nullptr;
  // Factored ordinate-form scatter G = L R^T (levels >= 1 whose K = (order+1)^2
  // harmonics are fewer than about A/2, where two GEMMs of 2AK flop per
  // spatial dof beat one of 2A^2): L (A x K), R (A x K), and the transposes
  // Lt, Rt (K x A); Kf = 0 when the dense G is used.
  int Kf = 0;
  double *L64 = nullptr, *R64 = nullptr, *Lt64 = nullptr, *Rt64 = nullptr;
  float *L32 = nullptr, *R32 = nullptr, *Lt32 = nullptr, *Rt32 = nullptr;
  // Octant-group form of the level scatter (levels >= 1 whose mesh is mapped
  // onto itself by the reflections of symR axes): Walsh-Hadamard blocks of
  // G, G^T and the canonical S~ ([2^symR][sym_nc][sym_ldb]) and the row map
  int symR = 0, sym_nc = 0, sym_ldb = 0;
  tr::OctMap om{};
  double *Bh64 = nullptr, *Bht64 = nullptr, *Bc64 = nullptr;
  float *Bh32 = nullptr, *Bht32 = nullptr, *Bc32 = nullptr;
  int *owner = nullptr;                    // level >= 1: owner patch on level l-1
  double *Pu = nullptr, *Ru = nullptr, *Pa = nullptr, *Ra = nullptr, *Pc = nullptr, *Rc = nullptr;
  int *first_child = nullptr, *n_child = nullptr;  // over level l-1 patches
  // workspaces (ordinate form); blk holds all of them, and on levels >= 1
  // the FP32 buffers are views of the same block
  double *blk = nullptr;
  double *f64 = nullptr, *u64 = nullptr, *sa64 = nullptr, *sb64 = nullptr;
  float *f32 = nullptr, *u32 = nullptr, *sa32 = nullptr, *sb32 = nullptr;
};

struct EventTimer {
  bool on = false;
  hipStream_t st = nullptr;
  struct Rec {
    int comp;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  int open_comp = -1;
  hipEvent_t open_ev = nullptr;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
  void begin(int comp) {
    if (!on) return;
    open_comp = comp;
    open_ev = get();
    HIPCHK(hipEventRecord(open_ev, st));
  }
  void end() {
    if (!on) return;
    hipEvent_t b = get();
    HIPCHK(hipEventRecord(b, st));
    recs.push_back({open_comp, open_ev, b});
  }
  ~EventTimer() {
    for (auto &r : recs) {
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
    }
    for (auto e : pool) hipEventDestroy(e);
  }
};

// Device scratch freed at scope exit (the caller synchronises the stream first).
struct TmpBuf {
  void *p = nullptr;
  explicit TmpBuf(size_t bytes) {
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) throw std::bad_alloc();
  }
  ~TmpBuf() { hipFree(p); }
  template <typename T>
  T *as() { return static_cast<T *>(p); }
};

enum { C_SWEEP = 0, C_SCATTER, C_TRANSFER, C_COARSE, C_APPLY, C_ORTH, C_OTHER, C_SWEEP_FINE, C_SCATTER_OUTER,
       C_SCATTER_FINE, C_N };

}  // namespace

struct tr_handle {
  tr_problem prob{};
  std::vector<double> sig_t_host, sig_s_host, moments;
  std::vector<int> mg_order;
  int octant_order[8];
  Grid g{};
  Planes pl{};
  std::vector<int> plane_off_host;
  std::vector<int> cells_host;    // the (+,+,+) sweep list (packed cells), plane by plane
  int *d_cells = nullptr, *d_off = nullptr;
  double *sig_t = nullptr, *sig_s = nullptr;
  double *sig_pl = nullptr;  // [2][8][cells] cross sections per orientation, cell-list order
  // brick schedule of the pair sweep (3-D, even cells along x), its slot
  // list (the cells brick by brick in sweep-frame order) and the cross
  // sections per orientation in slot order
  tr::Planes bpl{};
  int *d_slots = nullptr;
  double *sig_pb = nullptr;
  tr::HostAngular ang;
  std::vector<DevLevel> lv;
  double *Souter = nullptr;  // canonical S~ at the problem's order on the finest level
  double *Bouter = nullptr;  // its octant-group blocks (mesh with reflection structure), else null
  tr::OctMap outer_om{};
  int outer_R = 0, outer_nc = 0, outer_ldb = 0;
  double *iom = nullptr;     // [A][3] int Omega^xi psi on the finest level
  double *dot_partial = nullptr, *dot_out = nullptr;
  double *mdot_partial = nullptr, *mdot_out = nullptr;  // [32][dot_blocks], [2 m + 4]
  int mdot_len = 0;
  double *tmp = nullptr;     // one finest-level FP64 vector
  double *tmp2 = nullptr;
  int dot_blocks = 2048;
  // Krylov workspace
  int kry_m = 0;
  std::vector<double *> V, Z;
  std::vector<float *> Z32;       // FP32 preconditioned vectors (flexible form, FP32 preconditioners)
  bool dry = false;               // size-only setup (tr_workspace_bytes): nothing allocated or launched
  double *kw = nullptr, *kx = nullptr;
  bool mixed_ready = false;
  struct GsSchedule {
    int nu = 0;
    bool adj = false;
    int nsteps = 0, max_items = 0;
    int *step_off = nullptr, *items = nullptr;
    // dataflow form: per-wave slot lists (empty when not applicable)
    int waves = 0;
    int *wave_off = nullptr, *slots = nullptr;
    // brick form (3-D, even grids): one 2 x 2 x 2 brick per slot
    bool brick = false;
    long long nbricks = 0;
    int brick_steps = 0;
  };
  bool gs_brick = true;       // dataflow solve over 2 x 2 x 2 bricks where the grid allows
  bool split32 = false;       // FP32 scatter products from split-BF16 operands
  int *pos_pl = nullptr;      // [8][cells] position of a cell in each orientation's sweep list
  struct SplitA {             // level matrices split into BF16 hi/lo once
    const float *A;
    int M, K;
    void *p;
  };
  std::vector<SplitA> splits;
  bool gs_flow = true;        // coarse solve without grid barriers
  bool gs_coh = true;         // barrier form: device-coherent iterate accesses
  unsigned *gs_cnt = nullptr;  // [cells] update counters of the dataflow solve
  std::vector<GsSchedule> gs_sched;
  unsigned *bar_arrive = nullptr, *bar_release = nullptr;
  int *bar_err = nullptr;
  unsigned bar_gen = 0;
  static constexpr int kMaxGsBlocks = 1024;
  long long n_precond = 0;
  double sweep_dofs = 0;
  long long fact_len = 0;        // K x S of the largest factored level scatter
  double *fact64 = nullptr;      // R^T u (or L^T u) of a factored level
  float *fact32 = nullptr;
  int coarse_steps = 0;
  std::vector<void *> allocs;
  size_t bytes = 0;
  EventTimer *timer = nullptr;

  uintptr_t dry_next = 1 << 20;   // distinct stand-in addresses of a size-only setup (never dereferenced)
  template <typename T>
  T *alloc(size_t n) {
    void *p = nullptr;
    if (n == 0) n = 1;
    if (dry) {
      p = reinterpret_cast<void *>(dry_next);
      dry_next += (n * sizeof(T) + 255) / 256 * 256;
    } else {
      hipError_t e = hipMalloc(&p, n * sizeof(T));
      if (e != hipSuccess) throw std::bad_alloc();
      allocs.push_back(p);
    }
    bytes += n * sizeof(T);
    return static_cast<T *>(p);
  }
  template <typename T>
  T *upload(const std::vector<T> &v) {
    T *p = alloc<T>(v.size());
    if (!dry) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  int top() const { return (int)lv.size() - 1; }
  long long vec_len(int l) const { return (long long)lv[l].A * g.S; }
  ~tr_handle() {
    for (void *p : allocs) hipFree(p);  // empty for a size-only setup
  }
};

namespace {

void tbegin(tr_handle *h, int c) {
  if (h->timer) h->timer->begin(c);
}
void tend(tr_handle *h) {
  if (h->timer) h->timer->end();
}

// ------------------------------------------------------------------ setup
// Reflection structure of level l's mesh: the axes d whose reflection
// (sign flip of component d) maps every patch of octant o, at position k of
// that octant's list, onto the patch at position k of octant o ^ (1 << d),
// vertex by vertex.  Returns R = the number of such axes and fills urow
// ([2^R][nc]): transformed row t = (coset representative f, dof k within
// its octant) under sign pattern i (bit b of i = the b-th reflected axis)
// sits at canonical row urow[i * nc + t].
int octant_symmetry(const tr::HostAngular &ang, int l, std::vector<int> &urow, int &nc) {
  const tr::HostLevel &H = ang.lv[l];
  int first[8], cnt[8];
  for (int o = 0; o < 8; ++o) first[o] = -1, cnt[o] = 0;
  for (int q = 0; q < H.P; ++q) {
    const int o = H.octant[q];
    if (first[o] < 0) first[o] = q;
    else if (H.octant[q - 1] != o) return 0;  // not octant-major
    cnt[o]++;
  }
  int mask = 0;
  for (int d = 0; d < 3; ++d) {
    bool ok = true;
    for (int o = 0; o < 8 && ok; ++o) {
      const int o2 = o ^ (1 << d);
      if (cnt[o] != cnt[o2]) ok = false;
      for (int k = 0; k < cnt[o] && ok; ++k) {
        const tr::PatchNode &a = ang.tree[H.node[first[o] + k]], &b = ang.tree[H.node[first[o2] + k]];
        for (int v = 0; v < 3 && ok; ++v) {
          const double ax[3] = {a.v[v].x, a.v[v].y, a.v[v].z}, bx[3] = {b.v[v].x, b.v[v].y, b.v[v].z};
          for (int c = 0; c < 3; ++c)
            if (std::fabs((c == d ? -ax[c] : ax[c]) - bx[c]) > 1e-13) ok = false;
        }
      }
    }
    if (ok) mask |= 1 << d;
  }
  const int R = __builtin_popcount(mask);
  if (R == 0) return 0;
  int bits[3], nb = 0;
  for (int d = 0; d < 3; ++d)
    if (mask & (1 << d)) bits[nb++] = d;
  const int nchi = 1 << R;
  nc = H.A / nchi;
  urow.assign((size_t)nchi * nc, 0);
  int t = 0;
  for (int f = 0; f < 8; ++f) {
    if (f & mask) continue;  // coset representatives: reflected bits clear
    for (int k = 0; k < 3 * cnt[f]; ++k, ++t)
      for (int i = 0; i < nchi; ++i) {
        int o = f;
        for (int b = 0; b < R; ++b)
          if (i & (1 << b)) o |= 1 << bits[b];
        urow[(size_t)i * nc + t] = 3 * first[o] + k;
      }
  }
  if (t != nc) return 0;
  return R;
}

// The kernel's form of the row map: cosets as runs of transformed rows,
// canonical row = t + off[coset][i] (checked against urow).
tr::OctMap oct_map(const std::vector<int> &urow, int R, int nc) {
  tr::OctMap om{};
  om.R = R;
  om.nc = nc;
  const int nchi = 1 << R;
  // a new coset starts where the canonical row of pattern 0 jumps
  int c = 0;
  om.cstart[0] = 0;
  for (int t = 1; t < nc; ++t)
    if (urow[t] != urow[t - 1] + 1) {
      if (++c >= 8) throw std::runtime_error("internal: octant row map with more than 8 cosets");
      om.cstart[c] = t;
    }
  om.ncos = c + 1;
  for (int k = om.ncos; k <= 8; ++k) om.cstart[k] = nc;
  for (int k = 0; k < om.ncos; ++k)
    for (int i = 0; i < nchi; ++i) om.off[k][i] = urow[(size_t)i * nc + om.cstart[k]] - om.cstart[k];
  for (int k = 0; k < om.ncos; ++k)
    for (int t = om.cstart[k]; t < om.cstart[k + 1]; ++t)
      for (int i = 0; i < nchi; ++i)
        if (urow[(size_t)i * nc + t] != t + om.off[k][i]) throw std::runtime_error("internal: octant row map");
  if (om.ncos > (8 >> R)) throw std::runtime_error("internal: octant row map cosets");
  return om;
}

// Whether the A x A matrix M has the octant-group structure of urow:
// M[(i1, t1), (i2, t2)] = M[(0, t1), (i1 ^ i2, t2)] (checked on a sample of
// rows, to a relative 1e-12).
bool octant_structured(const std::vector<double> &M, int A, const std::vector<int> &urow, int R, int nc) {
  const int nchi = 1 << R;
  double mx = 0;
  for (double v : M) mx = std::max(mx, std::fabs(v));
  const int step = std::max(1, nc / 64);
  for (int t1 = 0; t1 < nc; t1 += step)
    for (int i1 = 0; i1 < nchi; ++i1)
      for (int i2 = 0; i2 < nchi; ++i2)
        for (int t2 = 0; t2 < nc; ++t2) {
          const double a = M[(size_t)urow[(size_t)i1 * nc + t1] * A + urow[(size_t)i2 * nc + t2]];
          const double b = M[(size_t)urow[t1] * A + urow[(size_t)(i1 ^ i2) * nc + t2]];
          if (std::fabs(a - b) > 1e-12 * mx) return false;
        }
  return true;
}

// Walsh-Hadamard blocks Bh[j][t1][t2] = 2^-R sum_i (-1)^{|i & j|} M[(0,t1),(i,t2)]
// with rows padded to ldb (zeros).
std::vector<double> octant_blocks(const std::vector<double> &M, int A, const std::vector<int> &urow, int R, int nc,
                                  int ldb) {
  const int nchi = 1 << R;
  std::vector<double> B((size_t)nchi * nc * ldb, 0.0);
  const double sc = 1.0 / nchi;
  for (int j = 0; j < nchi; ++j)
    for (int t1 = 0; t1 < nc; ++t1)
      for (int t2 = 0; t2 < nc; ++t2) {
        double v = 0;
        for (int i = 0; i < nchi; ++i) {
          const double m = M[(size_t)urow[t1] * A + urow[(size_t)i * nc + t2]];
          v += (__builtin_popcount(i & j) & 1) ? -m : m;
        }
        B[((size_t)j * nc + t1) * ldb + t2] = v * sc;
      }
  return B;
}

const tr_handle::GsSchedule &gs_schedule(tr_handle *h, int nu, bool adj);
void ensure_coarse_buffers(tr_handle *h);

// The slot list as a cell list (for the per-orientation cross-section tables).
tr::Planes slot_planes(const tr_handle *h) {
  tr::Planes sp{};
  sp.cells = h->d_slots;
  return sp;
}

void build(tr_handle *h, const tr_problem *p) {
  if (p->dim != 2 && p->dim != 3) throw ArgError{"dim must be 2 or 3"};
  for (int d = 0; d < p->dim; ++d) {
    if (p->n[d] < 1 || p->n[d] > 1000) throw ArgError{"cells per axis must be in 1..1000"};
    if (!(p->len[d] > 0)) throw ArgError{"domain lengths must be positive"};
  }
  if (p->order < 0 || p->order > 96) throw ArgError{"order out of range 0..96"};
  if (!p->moments || !p->sigma_t || !p->sigma_s || !p->mg_order) throw ArgError{"null array in problem"};
  if (p->nu_pre < 1 || p->nu_post < 0 || p->nu_coarse < 1 || p->nu_post_coarse < 0)
    throw ArgError{"need nu_pre >= 1, nu_post >= 0, nu_coarse >= 1, nu_post_coarse >= 0"};
  {
    int seen[8] = {0};
    for (int i = 0; i < 8; ++i) {
      int o = p->octant_order[i];
      if (o < 0 || o > 7 || seen[o]++) throw ArgError{"octant_order must be a permutation of 0..7"};
    }
  }
  h->prob = *p;
  std::memcpy(h->octant_order, p->octant_order, sizeof h->octant_order);
  Grid &g = h->g;
  g.dim = p->dim;
  g.ns = 1 << p->dim;
  g.n[0] = p->n[0];
  g.n[1] = p->n[1];
  g.n[2] = p->dim == 3 ? p->n[2] : 1;
  g.vol = 1.0;
  for (int d = 0; d < 3; ++d) {
    g.h[d] = d < p->dim ? p->len[d] / p->n[d] : 1.0;
    if (d < p->dim) g.vol *= g.h[d];
  }
  g.C = (long long)g.n[0] * g.n[1] * g.n[2];
  g.S = g.C * g.ns;
  h->sig_t_host.assign(p->sigma_t, p->sigma_t + g.C);
  h->sig_s_host.assign(p->sigma_s, p->sigma_s + g.C);
  for (long long j = 0; j < g.C; ++j) {
    if (!(std::isfinite(h->sig_t_host[j]) && h->sig_t_host[j] > 0)) throw ArgError{"sigma_t must be finite and > 0"};
    if (!(std::isfinite(h->sig_s_host[j]) && h->sig_s_host[j] >= 0)) throw ArgError{"sigma_s must be finite and >= 0"};
  }

  tr::RefineSpec spec;
  spec.base_level = p->ang_base_level;
  spec.cone_axis = {p->cone_axis[0], p->cone_axis[1], p->cone_axis[2]};
  spec.cone_half_angle_deg = p->cone_half_angle_deg;
  spec.cone_extra_levels = p->cone_extra_levels;
  spec.closure = p->irregularity_closure != 0;
  spec.band_lmax = p->band_lmax;
  if (p->angular_basis != TR_BASIS_LIN && p->angular_basis != TR_BASIS_CONST)
    throw ArgError{"angular_basis must be TR_BASIS_LIN or TR_BASIS_CONST"};
  spec.const_basis = p->angular_basis == TR_BASIS_CONST;
  if (spec.cone_extra_levels > 0 &&
      !(std::fabs(spec.cone_axis.x) + std::fabs(spec.cone_axis.y) + std::fabs(spec.cone_axis.z) > 0))
    throw ArgError{"cone axis must be nonzero"};
  std::string err;
  if (!tr::build_angular(spec, h->ang, err)) throw ArgError{err};
  const int nlev = (int)h->ang.lv.size();
  if (p->n_levels != nlev)
    throw ArgError{"n_levels does not match the angular mesh (it has " + std::to_string(nlev) + " levels)"};
  if (nlev > 16) throw ArgError{"too many angular levels"};
  h->mg_order.assign(p->mg_order, p->mg_order + nlev);
  int maxo = p->order;
  for (int o : h->mg_order) {
    if (o < 0 || o > 96) throw ArgError{"mg_order out of range 0..96"};
    maxo = std::max(maxo, o);
  }
  h->moments.assign(p->moments, p->moments + maxo + 1);
  for (double m : h->moments)
    if (!std::isfinite(m)) throw ArgError{"moments must be finite"};

  // sweep schedule (orientation +,+,+): cells grouped by ix + iy + iz
  {
    const int np = g.n[0] + g.n[1] + g.n[2] - 2;
    std::vector<std::vector<int>> buckets(np);
    for (int iz = 0; iz < g.n[2]; ++iz)
      for (int iy = 0; iy < g.n[1]; ++iy)
        for (int ix = 0; ix < g.n[0]; ++ix) buckets[ix + iy + iz].push_back(ix | (iy << 10) | (iz << 20));
    std::vector<int> cells, off{0};
    int mx = 0;
    for (auto &b : buckets) {
      cells.insert(cells.end(), b.begin(), b.end());
      off.push_back((int)cells.size());
      mx = std::max(mx, (int)b.size());
    }
    // positions of each cell's neighbours in the adjacent planes
    std::vector<int> pos(g.C);
    auto lin = [&](int ix, int iy, int iz) { return ix + (long long)g.n[0] * (iy + (long long)g.n[1] * iz); };
    for (int pl = 0; pl < np; ++pl)
      for (int i = off[pl]; i < off[pl + 1]; ++i) {
        const int c = cells[i];
        pos[lin(c & 1023, (c >> 10) & 1023, (c >> 20) & 1023)] = i - off[pl];
      }
    std::vector<int> link_up(4 * cells.size()), link_dn(4 * cells.size());
    for (size_t i = 0; i < cells.size(); ++i) {
      const int c = cells[i];
      const int ci[3] = {c & 1023, (c >> 10) & 1023, (c >> 20) & 1023};
      link_up[4 * i] = link_dn[4 * i] = c;
      for (int d = 0; d < 3; ++d) {
        int up = -1, dn = -1;
        if (d < g.dim) {
          int q[3] = {ci[0], ci[1], ci[2]};
          if (ci[d] > 0) {
            q[d] = ci[d] - 1;
            up = pos[lin(q[0], q[1], q[2])];
          }
          if (ci[d] < g.n[d] - 1) {
            q[d] = ci[d] + 1;
            dn = pos[lin(q[0], q[1], q[2])];
          }
        }
        link_up[4 * i + 1 + d] = up;
        link_dn[4 * i + 1 + d] = dn;
      }
    }
    h->pl.link[0] = reinterpret_cast<const int4 *>(h->upload(link_up));
    h->pl.link[1] = reinterpret_cast<const int4 *>(h->upload(link_dn));
    h->plane_off_host = off;
    h->cells_host = cells;
    // Brick schedule of the pair sweep: bricks of cells 2b, 2b + 1 along x
    // in the (+,+,+) frame, grouped by diagonal plane b + iy + iz, with the
    // positions of each brick's upwind bricks in the previous plane; the
    // slot list holds the cells brick by brick (slot 0 the upwind one).
    std::vector<int> slots;
    if (g.dim == 3 && g.n[0] % 2 == 0) {
      const int nb = g.n[0] / 2;
      const int npb = nb + g.n[1] + g.n[2] - 2;
      std::vector<std::vector<int>> bb(npb);
      for (int iz = 0; iz < g.n[2]; ++iz)
        for (int iy = 0; iy < g.n[1]; ++iy)
          for (int bx = 0; bx < nb; ++bx) bb[bx + iy + iz].push_back(bx | (iy << 10) | (iz << 20));
      std::vector<int> bricks, boff{0};
      int bmx = 0;
      for (auto &b : bb) {
        bricks.insert(bricks.end(), b.begin(), b.end());
        boff.push_back((int)bricks.size());
        bmx = std::max(bmx, (int)b.size());
      }
      std::vector<int> bpos((size_t)nb * g.n[1] * g.n[2]);
      auto blin = [&](int bx, int iy, int iz) { return bx + (long long)nb * (iy + (long long)g.n[1] * iz); };
      for (int pl = 0; pl < npb; ++pl)
        for (int i = boff[pl]; i < boff[pl + 1]; ++i) {
          const int c = bricks[i];
          bpos[blin(c & 1023, (c >> 10) & 1023, (c >> 20) & 1023)] = i - boff[pl];
        }
      std::vector<int> blink(4 * bricks.size());
      slots.resize(2 * bricks.size());
      for (size_t i = 0; i < bricks.size(); ++i) {
        const int c = bricks[i];
        const int ci[3] = {c & 1023, (c >> 10) & 1023, (c >> 20) & 1023};
        blink[4 * i] = c;
        for (int d = 0; d < 3; ++d) {
          int q[3] = {ci[0], ci[1], ci[2]};
          int up = -1;
          if (ci[d] > 0) {
            q[d] = ci[d] - 1;
            up = bpos[blin(q[0], q[1], q[2])];
          }
          blink[4 * i + 1 + d] = up;
        }
        for (int sl = 0; sl < 2; ++sl) slots[2 * i + sl] = (2 * ci[0] + sl) | (ci[1] << 10) | (ci[2] << 20);
      }
      h->bpl.cells = h->upload(bricks);
      h->bpl.off = h->upload(boff);
      h->bpl.nplanes = npb;
      h->bpl.max_plane = bmx;
      h->bpl.link[0] = reinterpret_cast<const int4 *>(h->upload(blink));
      h->bpl.link[1] = nullptr;
      h->d_slots = h->upload(slots);
    }
    // position of every cell in each orientation's sweep list (the plane
    // layout of forward sweep inputs): the cell list, or with the pair
    // sweep the slot list
    {
      const std::vector<int> &order = slots.empty() ? cells : slots;
      std::vector<int> ppos(8 * (size_t)g.C);
      for (int fl = 0; fl < 8; ++fl)
        for (size_t i = 0; i < order.size(); ++i) {
          const int c = order[i];
          int ix[3] = {c & 1023, (c >> 10) & 1023, (c >> 20) & 1023};
          for (int d = 0; d < 3; ++d)
            if ((fl >> d) & 1) ix[d] = g.n[d] - 1 - ix[d];
          ppos[(size_t)fl * g.C + lin(ix[0], ix[1], ix[2])] = (int)i;
        }
      h->pos_pl = h->upload(ppos);
    }
    h->d_cells = h->upload(cells);
    h->d_off = h->upload(off);
    h->pl.cells = h->d_cells;
    h->pl.off = h->d_off;
    h->pl.nplanes = np;
    h->pl.max_plane = mx;
  }
  h->sig_t = h->upload(h->sig_t_host);
  h->sig_s = h->upload(h->sig_s_host);
  h->sig_pl = h->alloc<double>(16 * g.C);
  if (h->d_slots) h->sig_pb = h->alloc<double>(16 * g.C);
  if (!h->dry) {
    tr::launch_sigma_planes(h->sig_t, h->sig_s, h->pl, g, h->sig_pl, nullptr);
    if (h->d_slots) tr::launch_sigma_planes(h->sig_t, h->sig_s, slot_planes(h), g, h->sig_pb, nullptr);
    HIPCHK(hipDeviceSynchronize());
  }

  // levels
  h->lv.assign(nlev, DevLevel());
  for (int l = 0; l < nlev; ++l) {
    const tr::HostLevel &H = h->ang.lv[l];
    DevLevel &D = h->lv[l];
    D.P = H.P;
    D.A = H.A;
    D.order = h->mg_order[l];
    std::vector<OrdInfo> ord(H.A);
    std::vector<double> winv(H.A);
    for (int a = 0; a < H.A; ++a) {
      OrdInfo o{};
      int flip = 0;
      for (int d = 0; d < 3; ++d) {
        double om = H.omega[3 * a + d];
        bool active = d < g.dim;
        o.a[d] = active ? std::fabs(om) : 0.0;
        o.c[d] = active ? std::fabs(om) / g.h[d] : 0.0;
        if (active && om < 0) flip |= 1 << d;
      }
      o.flip = flip;
      o.patch = a / 3;
      ord[a] = o;
      if (!(H.w[a] > 0)) throw ArgError{"internal: nonpositive quadrature weight"};
      winv[a] = 1.0 / H.w[a];
    }
    // the three ordinates of a patch sweep in one orientation (the operator
    // apply, the plane-layout transfers and the coarse solve rely on it;
    // octant-contained patches guarantee it)
    for (int a = 0; a + 2 < H.A; a += 3)
      if (ord[a].flip != ord[a + 1].flip || ord[a].flip != ord[a + 2].flip)
        throw std::runtime_error("internal: ordinates of one patch in different orientations");
    D.ord = h->upload(ord);
    // forward sweep inputs in plane layout on the V-cycle's smoothing levels
    // when their sweeps run in the LDS kernel (one pre-smoothing sweep: the
    // restricted residual then needs no plane-layout input)
    // with the pair sweep the plane layout is its slot order, read by no
    // other kernel
    const bool pairs = h->bpl.nplanes > 0;
    D.pin64 = l >= 1 && l < nlev && h->prob.nu_pre == 1 &&
              (pairs ? tr::sweep_pair_fits<double>(h->bpl) : tr::sweep_lds_fits<double>(h->pl, g, false));
    D.pin32 = l >= 1 && l < nlev && h->prob.nu_pre == 1 &&
              (pairs ? tr::sweep_pair_fits<float>(h->bpl) : tr::sweep_lds_fits<float>(h->pl, g, false));
    D.w = h->upload(H.w);
    D.winv = h->upload(winv);
    D.ipsi = h->upload(H.ipsi);
    // scatter matrices at this level's order
    std::vector<double> mom(h->moments.begin(), h->moments.begin() + D.order + 1);
    std::vector<double> St, X;
    tr::scatter_matrix(h->ang, l, mom, St, &X);
    const int A = H.A;
    const int K = (D.order + 1) * (D.order + 1);
    // scatter form of levels >= 1, by multiply-adds per spatial dof: the
    // octant-group blocks (2 A^2 / 2^R) where the mesh has the reflection
    // structure, the factored form (4 A K) where K is small, else dense
    std::vector<int> urow;
    int nc = 0;
    const int R = l >= 1 ? octant_symmetry(h->ang, l, urow, nc) : 0;
    const double cost_sym = R ? 2.0 * A * A / (1 << R) : 1e300;
    if (l >= 1 && 20LL * K < 9LL * A && 4.0 * A * K < cost_sym) {
      // G = L R^T with L_q = W_q^{-1} Psi^{-1} X_q F and R_p = Psi^{-1} X_p
      std::vector<double> Lh((size_t)A * K), Rh((size_t)A * K), Lt((size_t)K * A), Rt((size_t)K * A);
      for (int q = 0; q < H.P; ++q)
        for (int k = 0; k < 3; ++k)
          for (int c = 0; c < K; ++c) {
            const int n = (int)std::floor(std::sqrt((double)c) + 1e-9);
            double r = 0.0;
            for (int m = 0; m < 3; ++m) r += kPsiInv[k][m] * X[(size_t)(3 * q + m) * K + c];
            const int a = 3 * q + k;
            Rh[(size_t)a * K + c] = r;
            Rt[(size_t)c * A + a] = r;
            const double lv = r * mom[n] / H.w[a];
            Lh[(size_t)a * K + c] = lv;
            Lt[(size_t)c * A + a] = lv;
          }
      D.Kf = K;
      D.L64 = h->upload(Lh);
      D.R64 = h->upload(Rh);
      D.Lt64 = h->upload(Lt);
      D.Rt64 = h->upload(Rt);
      std::vector<float> l32(Lh.begin(), Lh.end()), r32(Rh.begin(), Rh.end()), lt32(Lt.begin(), Lt.end()),
          rt32(Rt.begin(), Rt.end());
      D.L32 = h->upload(l32);
      D.R32 = h->upload(r32);
      D.Lt32 = h->upload(lt32);
      D.Rt32 = h->upload(rt32);
      h->fact_len = std::max(h->fact_len, (long long)K * g.S);
    }
    std::vector<double> G((size_t)A * A), Gt((size_t)A * A);
    for (int q = 0; q < H.P; ++q)
      for (int p2 = 0; p2 < H.P; ++p2) {
        double blk[9], t1[9], t2[9];
        for (int m = 0; m < 3; ++m)
          for (int d = 0; d < 3; ++d) blk[m * 3 + d] = St[(size_t)(3 * q + m) * A + 3 * p2 + d];
        mat3_mul(&kPsiInv[0][0], blk, t1);
        mat3_mul(t1, &kPsiInv[0][0], t2);
        for (int k = 0; k < 3; ++k)
          for (int kk = 0; kk < 3; ++kk) {
            double v = t2[k * 3 + kk] / H.w[3 * q + k];
            G[(size_t)(3 * q + k) * A + 3 * p2 + kk] = v;
            Gt[(size_t)(3 * p2 + kk) * A + 3 * q + k] = v;
          }
      }
    if (R && !D.Kf && octant_structured(G, A, urow, R, nc) && octant_structured(Gt, A, urow, R, nc) &&
        octant_structured(St, A, urow, R, nc)) {
      D.symR = R;
      D.sym_nc = nc;
      D.sym_ldb = (nc + 3) / 4 * 4;
      D.om = oct_map(urow, R, nc);
      auto up2 = [&](const std::vector<double> &M, double *&b64, float *&b32) {
        std::vector<double> B = octant_blocks(M, A, urow, R, nc, D.sym_ldb);
        b64 = h->upload(B);
        b32 = h->upload(std::vector<float>(B.begin(), B.end()));
      };
      up2(G, D.Bh64, D.Bh32);
      up2(Gt, D.Bht64, D.Bht32);
      up2(St, D.Bc64, D.Bc32);
    }
    std::vector<float> St32(St.begin(), St.end()), G32(G.begin(), G.end()), Gt32(Gt.begin(), Gt.end());
    D.St64 = h->upload(St);
    D.St32 = h->upload(St32);
    D.G64 = h->upload(G);
    D.Gt64 = h->upload(Gt);
    D.G32 = h->upload(G32);
    D.Gt32 = h->upload(Gt32);
    if (l == nlev - 1) {
      if (p->order == D.order) {
        h->Souter = D.St64;
        h->Bouter = D.Bc64;
      } else {
        std::vector<double> mo(h->moments.begin(), h->moments.begin() + p->order + 1), So;
        tr::scatter_matrix(h->ang, l, mo, So);
        h->Souter = h->upload(So);
        std::vector<int> ur;
        int ncc = 0;
        const int Ro = l >= 1 ? octant_symmetry(h->ang, l, ur, ncc) : 0;
        if (Ro && octant_structured(So, A, ur, Ro, ncc)) {
          h->outer_om = oct_map(ur, Ro, ncc);
          h->outer_R = Ro;
          h->outer_nc = ncc;
          h->outer_ldb = (ncc + 3) / 4 * 4;
          h->Bouter = h->upload(octant_blocks(So, A, ur, Ro, ncc, h->outer_ldb));
        }
      }
      if (h->Bouter && !h->outer_R) {
        h->outer_om = D.om;
        h->outer_R = D.symR;
        h->outer_nc = D.sym_nc;
        h->outer_ldb = D.sym_ldb;
      }
      h->iom = h->upload(H.iom);
    }
    if (l > 0) {
      const tr::HostLevel &Hc = h->ang.lv[l - 1];
      std::vector<double> Pu(9 * (size_t)H.P), Ru(9 * (size_t)H.P), Pa(9 * (size_t)H.P), Ra(9 * (size_t)H.P),
          Pc(9 * (size_t)H.P), Rc(9 * (size_t)H.P);
      for (int c = 0; c < H.P; ++c) {
        const int par = H.owner[c];
        double P0[9], PT[9], t1[9], t2[9];
        for (int i = 0; i < 9; ++i) P0[i] = H.pblk[(size_t)c * 9 + i];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) PT[i * 3 + j] = P0[j * 3 + i];
        double Wc[9] = {0}, Wpi[9] = {0};
        for (int k = 0; k < 3; ++k) {
          Wc[k * 4] = H.w[3 * c + k];
          Wpi[k * 4] = 1.0 / Hc.w[3 * par + k];
        }
        // ordinate-form prolongation  Psi P Psi^{-1}
        mat3_mul(&kPsi[0][0], P0, t1);
        mat3_mul(t1, &kPsiInv[0][0], t2);
        std::memcpy(&Pu[9 * (size_t)c], t2, sizeof t2);
        // ordinate-form restriction  W_p^{-1} Psi^{-1} P^T Psi W_c
        mat3_mul(Wpi, &kPsiInv[0][0], t1);
        mat3_mul(t1, PT, t2);
        mat3_mul(t2, &kPsi[0][0], t1);
        mat3_mul(t1, Wc, t2);
        std::memcpy(&Ru[9 * (size_t)c], t2, sizeof t2);
        // adjoint form: prolongation W_c Psi P Psi^{-1} W_p^{-1}
        mat3_mul(Wc, &kPsi[0][0], t1);
        mat3_mul(t1, P0, t2);
        mat3_mul(t2, &kPsiInv[0][0], t1);
        mat3_mul(t1, Wpi, t2);
        std::memcpy(&Pa[9 * (size_t)c], t2, sizeof t2);
        // adjoint form: restriction Psi^{-1} P^T Psi
        mat3_mul(&kPsiInv[0][0], PT, t1);
        mat3_mul(t1, &kPsi[0][0], t2);
        std::memcpy(&Ra[9 * (size_t)c], t2, sizeof t2);
        std::memcpy(&Pc[9 * (size_t)c], P0, sizeof P0);
        std::memcpy(&Rc[9 * (size_t)c], PT, sizeof PT);
      }
      D.owner = h->upload(H.owner);
      D.Pu = h->upload(Pu);
      D.Ru = h->upload(Ru);
      D.Pa = h->upload(Pa);
      D.Ra = h->upload(Ra);
      D.Pc = h->upload(Pc);
      D.Rc = h->upload(Rc);
      D.first_child = h->upload(H.first_child);
      D.n_child = h->upload(H.n_child);
    }
    // level buffers f, u, s (and a second s for nu_pre > 1) in one block;
    // on levels >= 1 the FP32 V-cycle's buffers live in the same memory
    // (a solve uses one precision per level at a time)
    const long long n = (long long)D.A * g.S;
    const int nbuf = p->nu_pre > 1 ? 4 : 3;
    D.blk = h->alloc<double>(nbuf * n);
    D.f64 = D.blk;
    D.u64 = D.blk + n;
    D.sa64 = D.blk + 2 * n;
    D.sb64 = p->nu_pre > 1 ? D.blk + 3 * n : nullptr;
    if (!h->dry) {
      tr::launch_fill<double>(D.f64, n, 0.0, nullptr);
      tr::launch_fill<double>(D.u64, n, 0.0, nullptr);
    }
  }
  if (h->fact_len > 0) h->fact64 = h->alloc<double>(h->fact_len);
  const long long nf = h->vec_len(h->top());
  h->tmp = h->alloc<double>(nf);
  h->tmp2 = h->alloc<double>(nf);
  h->dot_partial = h->alloc<double>(h->dot_blocks);
  h->dot_out = h->alloc<double>(1);
  // the coarse solve's schedules for nu_coarse sweeps (both directions) and
  // its counters, so that no solve or coarse-solve call allocates them
  gs_schedule(h, p->nu_coarse, false);
  gs_schedule(h, p->nu_coarse, true);
  ensure_coarse_buffers(h);
  if (!h->dry) HIPCHK(hipDeviceSynchronize());
}

void ensure_mixed(tr_handle *h) {
  if (h->mixed_ready) return;
  for (int l = 1; l < (int)h->lv.size(); ++l) {
    DevLevel &D = h->lv[l];
    const long long n = (long long)D.A * h->g.S;
    // FP32 views of the level block (see build)
    float *b32 = reinterpret_cast<float *>(D.blk);
    D.f32 = b32;
    D.u32 = b32 + n;
    D.sa32 = b32 + 2 * n;
    D.sb32 = h->prob.nu_pre > 1 ? b32 + 3 * n : nullptr;
  }
  if (h->fact_len > 0) h->fact32 = h->alloc<float>(h->fact_len);
  h->mixed_ready = true;
}

// --------------------------------------------------------------- pieces
template <typename T>
struct LevelBuf;
template <>
struct LevelBuf<double> {
  static double *fact(tr_handle *h) { return h->fact64; }
  static const double *Lf(DevLevel &D, bool adj) { return adj ? D.Lt64 : D.Rt64; }  // first factor (K x A)
  static const double *Rf(DevLevel &D, bool adj) { return adj ? D.R64 : D.L64; }   // second factor (A x K)
  static double *f(DevLevel &D) { return D.f64; }
  static double *u(DevLevel &D) { return D.u64; }
  static double *sa(DevLevel &D) { return D.sa64; }
  static double *sb(DevLevel &D) { return D.sb64; }
  static const double *G(DevLevel &D, bool adj) { return adj ? D.Gt64 : D.G64; }
  static const double *St(DevLevel &D) { return D.St64; }
  static const double *Bh(DevLevel &D, bool adj) { return adj ? D.Bht64 : D.Bh64; }
  static bool pin(const DevLevel &D) { return D.pin64; }
  static const double *Bc(DevLevel &D) { return D.Bc64; }
};
template <>
struct LevelBuf<float> {
  static float *fact(tr_handle *h) { return h->fact32; }
  static const float *Lf(DevLevel &D, bool adj) { return adj ? D.Lt32 : D.Rt32; }
  static const float *Rf(DevLevel &D, bool adj) { return adj ? D.R32 : D.L32; }
  static float *f(DevLevel &D) { return D.f32; }
  static float *u(DevLevel &D) { return D.u32; }
  static float *sa(DevLevel &D) { return D.sa32; }
  static float *sb(DevLevel &D) { return D.sb32; }
  static const float *G(DevLevel &D, bool adj) { return adj ? D.Gt32 : D.G32; }
  static const float *St(DevLevel &D) { return D.St32; }
  static const float *Bh(DevLevel &D, bool adj) { return adj ? D.Bht32 : D.Bh32; }
  static bool pin(const DevLevel &D) { return D.pin32; }
  static const float *Bc(DevLevel &D) { return D.Bc32; }
};

template <typename T>
void do_sweep(tr_handle *h, int l, const T *f, const T *s, T *u, bool adj, hipStream_t st) {
  tr::SweepArgs<T> a;
  a.f = f;
  a.s = s;
  a.u = u;
  a.sig_t = h->sig_t;
  a.sig_s = h->sig_s;
  a.sig_pl = h->sig_pl;
  a.ord = h->lv[l].ord;
  a.pl = h->pl;
  a.g = h->g;
  a.plane_in = !adj && (sizeof(T) == 8 ? h->lv[l].pin64 : h->lv[l].pin32);
  a.bpl = h->bpl;
  a.sig_pb = h->sig_pb;
  const bool fine = l == h->top();
  h->sweep_dofs += (double)h->lv[l].A * (double)h->g.S;
  tbegin(h, fine ? C_SWEEP_FINE : C_SWEEP);
  tr::launch_sweep<T>(a, h->lv[l].A, adj, st);
  tend(h);
}

// The split-BF16 form of a constant level matrix (made on first use).
const void *split_of(tr_handle *h, const float *A, int M, int K, hipStream_t st) {
  for (auto &e : h->splits)
    if (e.A == A && e.M == M && e.K == K) return e.p;
  void *p = h->alloc<unsigned short>(2LL * M * tr::split_rows_kp(K));
  if (!h->dry) tr::launch_split_rows(A, M, K, p, st);
  h->splits.push_back({A, M, K, p});
  return p;
}

// The split-BF16 form of a level's octant-group blocks Bh ([2^R nc][ldb]).
const void *split_blocks(tr_handle *h, const DevLevel &D, const float *Bh, hipStream_t st) {
  return split_of(h, Bh, (1 << D.symR) * D.sym_nc, D.sym_ldb, st);
}

// C = A B on the level GEMM path: FP64 and FP32 on the matrix cores in
// their own precision, FP32 from split-BF16 operands when the handle's
// preconditioner mode asks for it.
template <typename T>
void gemm(tr_handle *h, const T *A, const T *B, T *C, int M, int N, int K, hipStream_t st, const T *bias = nullptr,
          const double *colscale = nullptr, int cell = 8, const int *pos = nullptr, const OrdInfo *rord = nullptr) {
  if constexpr (std::is_same<T, float>::value) {
    if (h->split32) {
      tr::launch_gemm_bf16x3(split_of(h, A, M, K, st), B, C, M, N, K, st, bias, colscale, cell, pos, rord);
      return;
    }
  }
  tr::launch_gemm<T>(A, B, C, M, N, K, st, bias, colscale, cell, pos, rord);
}

// y = G x, or y = bias + sigma_s (G x) per cell with scale_sn (bias may be
// null): the forward V-cycle's prepared right-hand sides; with rord the
// result (and the bias) are in plane layout for the level's ordinates.
template <typename T>
void do_gemm(tr_handle *h, const T *G, const T *x, T *y, int A, hipStream_t st, bool scale_sn = false,
             const T *bias = nullptr, const OrdInfo *rord = nullptr, int comp = C_SCATTER) {
  tbegin(h, comp);
  gemm<T>(h, G, x, y, A, (int)h->g.S, A, st, bias, scale_sn ? h->sig_s : nullptr, h->g.ns,
          rord ? h->pos_pl : nullptr, rord);
  tend(h);
}

// Step schedule of nu Gauss-Seidel sweeps on T_0 (octants in the given
// order, cells in upwind order, downwind first for the adjoint): each
// (sweep, octant, cell) update goes one step after the latest of its
// upwind neighbours' updates in the same octant sweep and of the cell's
// previous update, the earliest step at which everything it reads is final.
const tr_handle::GsSchedule &gs_schedule(tr_handle *h, int nu, bool adj) {
  for (auto &sc : h->gs_sched)
    if (sc.nu == nu && sc.adj == adj) return sc;
  const Grid &g = h->g;
  const long long C = g.C;
  std::vector<int> last(C, -1), to(C, -1);
  std::vector<std::vector<int>> steps, fsteps;
  const int np = h->pl.nplanes;
  const std::vector<int> &cells_host = h->cells_host;
  const bool flow_ok = 8 * nu <= 127 && C < (1LL << 22);
  for (int sweep = 0; sweep < nu; ++sweep)
    for (int oi = 0; oi < 8; ++oi) {
      const int o = h->octant_order[oi];
      const int cnt_before = 8 * sweep + oi;  // updates every cell has had before this octant sweep
      for (int pp = 0; pp < np; ++pp) {
        const int p = adj ? np - 1 - pp : pp;
        for (int idx = h->plane_off_host[p]; idx < h->plane_off_host[p + 1]; ++idx) {
          const int packed = cells_host[idx];
          int ci[3] = {packed & 1023, (packed >> 10) & 1023, (packed >> 20) & 1023}, ix[3];
          for (int d = 0; d < 3; ++d) ix[d] = ((o >> d) & 1) ? g.n[d] - 1 - ci[d] : ci[d];
          const long long j = ix[0] + (long long)g.n[0] * (ix[1] + (long long)g.n[1] * ix[2]);
          int t = last[j] + 1;
          for (int d = 0; d < g.dim; ++d) {
            const bool has = adj ? ci[d] < g.n[d] - 1 : ci[d] > 0;
            if (!has) continue;
            int nx[3] = {ix[0], ix[1], ix[2]};
            const int dir = ((o >> d) & 1) ? -1 : 1;
            nx[d] += adj ? dir : -dir;
            const long long jn = nx[0] + (long long)g.n[0] * (nx[1] + (long long)g.n[1] * nx[2]);
            t = std::max(t, to[jn] + 1);
          }
          to[j] = t;
          last[j] = t;
          if ((int)steps.size() <= t) {
            steps.resize(t + 1);
            fsteps.resize(t + 1);
          }
          steps[t].push_back((o << 28) | idx);
          if (flow_ok) fsteps[t].push_back((int)(((unsigned)o << 29) | ((unsigned)cnt_before << 22) | (unsigned)idx));
        }
      }
    }
  std::vector<int> off{0}, items;
  int mx = 0;
  for (auto &st : steps) {
    items.insert(items.end(), st.begin(), st.end());
    off.push_back((int)items.size());
    mx = std::max(mx, (int)st.size());
  }
  tr_handle::GsSchedule sc;
  sc.nu = nu;
  sc.adj = adj;
  sc.nsteps = (int)steps.size();
  sc.max_items = mx;
  sc.step_off = h->upload(off);
  sc.items = h->upload(items);
  if (flow_ok) {
    // slots of 64 / 2^dim updates dealt round-robin to the waves, step by
    // step, so every wave's list is in step order.  Four waves per slot of
    // the widest step: a wave is busy with one slot for about four steps
    // (waits, coherent loads, store acknowledgement), measured best on the
    // 32^3 problem (512 waves: 12.2 ms per 10-sweep solve; 256: 13.0;
    // 1024: 12.6); at most 1024 waves, which stay co-resident.
    const int per = 64 / g.ns;
    const int W = 4 * std::max(1, std::min(256, (mx + per - 1) / per));
    std::vector<std::vector<int>> lists(W);
    int next = 0;
    for (auto &st : fsteps)
      for (size_t i0 = 0; i0 < st.size(); i0 += per) {
        auto &L = lists[next];
        for (int k = 0; k < per; ++k) L.push_back(i0 + k < st.size() ? st[i0 + k] : -1);
        next = (next + 1) % W;
      }
    std::vector<int> woff{0}, sl;
    for (auto &L : lists) {
      sl.insert(sl.end(), L.begin(), L.end());
      woff.push_back((int)(sl.size() / per));
    }
    sc.waves = W;
    sc.wave_off = h->upload(woff);
    sc.slots = h->upload(sl);
  }
  if (flow_ok && h->gs_brick && g.dim == 3 && !((g.n[0] | g.n[1] | g.n[2]) & 1)) {
    // the same schedule on the grid of 2 x 2 x 2 bricks, in each sweep's
    // direction (the adjoint's sweeps run the other way).
    const int nb[3] = {g.n[0] / 2, g.n[1] / 2, g.n[2] / 2};
    const long long NB = (long long)nb[0] * nb[1] * nb[2];
    std::vector<std::array<int, 3>> pbs;
    for (int z = 0; z < nb[2]; ++z)
      for (int y = 0; y < nb[1]; ++y)
        for (int x = 0; x < nb[0]; ++x) pbs.push_back({x, y, z});
    std::stable_sort(pbs.begin(), pbs.end(), [](const std::array<int, 3> &a, const std::array<int, 3> &b) {
      return a[0] + a[1] + a[2] < b[0] + b[1] + b[2];
    });
    auto bidx = [&](const int *bx) { return bx[0] + (long long)nb[0] * (bx[1] + (long long)nb[1] * bx[2]); };
    std::vector<int> lastb(NB, -1);
    std::vector<std::vector<int>> bsteps;
    for (int sweep = 0; sweep < nu; ++sweep)
      for (int oi = 0; oi < 8; ++oi) {
        const int o = h->octant_order[oi];
        const unsigned c = 8u * sweep + oi;
        for (auto &pb : pbs) {
          int bx[3];
          bool rev[3];
          for (int d = 0; d < 3; ++d) {
            rev[d] = (((o >> d) & 1) != 0) != adj;
            bx[d] = rev[d] ? nb[d] - 1 - pb[d] : pb[d];
          }
          const long long B = bidx(bx);
          int t = lastb[B] + 1;
          for (int d = 0; d < 3; ++d) {
            if (pb[d] == 0) continue;
            int by[3] = {bx[0], bx[1], bx[2]};
            by[d] += rev[d] ? 1 : -1;
            t = std::max(t, lastb[bidx(by)] + 1);
          }
          lastb[B] = t;
          if ((int)bsteps.size() <= t) bsteps.resize(t + 1);
          bsteps[t].push_back((int)(((unsigned)o << 29) | (c << 22) | (unsigned)B));
        }
      }
    int bmx = 0;
    for (auto &st : bsteps) bmx = std::max(bmx, (int)st.size());
    // two slot lists (one workgroup of three waves each) per brick of the
    // widest step, as many as stay co-resident (four per CU on MI355X: 1024;
    // assumed without a device).  A list works its slots one after the
    // other, so fewer lists lengthen the solve: 32^3 problem (widest step
    // 256 bricks), 10 sweeps, 5.0 ms with 512 lists, 11.6 ms with 256; 48^3
    // (widest step 576) 13.7 ms with 512 lists, 10.1 ms with 1024
    static const int capacity = tr::coarse_brick_capacity();
    const int cap = capacity > 0 ? capacity : 1024;
    const int W = 2 * std::max(2, std::min(cap / 2, bmx));
    std::vector<std::vector<int>> lists(W);
    int next = 0;
    for (auto &st : bsteps)
      for (int it : st) {
        lists[next].push_back(it);
        next = (next + 1) % W;
      }
    std::vector<int> woff{0}, sl;
    for (auto &L : lists) {
      sl.insert(sl.end(), L.begin(), L.end());
      woff.push_back((int)sl.size());
    }
    sc.brick = true;
    sc.nbricks = NB;
    sc.brick_steps = (int)bsteps.size();
    sc.waves = W;
    sc.wave_off = h->upload(woff);
    sc.slots = h->upload(sl);
  }
  h->gs_sched.push_back(sc);
  return h->gs_sched.back();
}

// After a coarse solve: a wait that timed out set the error word; it is
// cleared again (the handle stays usable) and the call reports the error.
void check_barrier(tr_handle *h, hipStream_t st) {
  if (!h->bar_err) return;
  int e = 0;
  HIPCHK(hipMemcpyAsync(&e, h->bar_err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (e) {
    HIPCHK(hipMemset(h->bar_err, 0, sizeof(int)));
    HIPCHK(hipDeviceSynchronize());
    throw std::runtime_error("coarse Gauss-Seidel solve timed out waiting for a grid barrier or an upwind update");
  }
}

// Barrier words, the error word and the update counters of the coarse
// solve (allocated once per handle).
void ensure_coarse_buffers(tr_handle *h) {
  if (!h->bar_arrive) {
    h->bar_arrive = h->alloc<unsigned>(tr_handle::kMaxGsBlocks);
    h->bar_release = h->alloc<unsigned>(1);
    h->bar_err = h->alloc<int>(1);
    if (!h->dry) {
      HIPCHK(hipMemset(h->bar_arrive, 0, tr_handle::kMaxGsBlocks * sizeof(unsigned)));
      HIPCHK(hipMemset(h->bar_release, 0, sizeof(unsigned)));
      HIPCHK(hipMemset(h->bar_err, 0, sizeof(int)));
      HIPCHK(hipDeviceSynchronize());
    }
    h->bar_gen = 0;
  }
  if (h->gs_flow && !h->gs_cnt) h->gs_cnt = h->alloc<unsigned>(h->g.C);
}

void do_coarse(tr_handle *h, const double *f, double *u, int nu, bool adj, hipStream_t st) {
  DevLevel &D = h->lv[0];
  const tr_handle::GsSchedule &sc = gs_schedule(h, nu, adj);
  ensure_coarse_buffers(h);
  if (h->bar_gen > 0xF0000000u - (unsigned)sc.nsteps) {
    // restart the generation count (all earlier launches on this handle's
    // stream have finished once the stream is synchronised)
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemset(h->bar_arrive, 0, tr_handle::kMaxGsBlocks * sizeof(unsigned)));
    HIPCHK(hipMemset(h->bar_release, 0, sizeof(unsigned)));
    HIPCHK(hipDeviceSynchronize());
    h->bar_gen = 0;
  }
  if (h->gs_flow && sc.brick) {
    tbegin(h, C_COARSE);
    tr::launch_coarse_brick(f, u, adj ? D.Gt64 : D.G64, h->sig_t, h->sig_s, D.ord, h->g, sc.wave_off, sc.slots,
                            sc.waves, adj, h->gs_cnt, sc.nbricks, h->bar_err, st);
    tend(h);
    h->coarse_steps = sc.brick_steps;
    return;
  }
  if (h->gs_flow && sc.waves > 0) {
    tbegin(h, C_COARSE);
    tr::launch_coarse_flow(f, u, adj ? D.Gt64 : D.G64, h->sig_t, h->sig_s, D.ord, h->pl, h->g, sc.wave_off,
                           sc.slots, sc.waves, adj, h->gs_cnt, h->bar_err, st);
    tend(h);
    h->coarse_steps = sc.nsteps;
    return;
  }
  tbegin(h, C_COARSE);
  tr::launch_coarse_gs(f, u, adj ? D.Gt64 : D.G64, h->sig_t, h->sig_s, D.ord, h->pl, h->g, sc.step_off, sc.items,
                       sc.nsteps, sc.max_items, adj, h->bar_arrive, h->bar_release, h->bar_err,
                       tr_handle::kMaxGsBlocks, h->bar_gen, h->gs_coh, st);
  tend(h);
  h->bar_gen += (unsigned)sc.nsteps;
  h->coarse_steps = sc.nsteps;
}

// Level scatter y = G_l u (transpose for the adjoint), with the forward
// epilogue of do_gemm; factored levels take two GEMMs through a K x S
// intermediate: G u = L (R^T u), G^T u = R (L^T u).
template <typename T>
void level_scatter(tr_handle *h, int l, bool adj, const T *u, T *y, hipStream_t st, bool scale_sn = false,
                   const T *bias = nullptr, bool plane_out = false) {
  DevLevel &D = h->lv[l];
  const OrdInfo *rord = plane_out ? D.ord : nullptr;
  const int comp = l == h->top() ? C_SCATTER_FINE : C_SCATTER;  // timer component
  if (D.symR) {
    // octant-group blocks
    tbegin(h, comp);
    bool done = false;
    if constexpr (std::is_same<T, float>::value) {
      if (h->split32) {
        tr::launch_gemm_oct_bf16x3(split_blocks(h, D, LevelBuf<T>::Bh(D, adj), st), tr::split_rows_kp(D.sym_ldb), u,
                                   y, D.om, (int)h->g.S, st, bias, scale_sn ? h->sig_s : nullptr, h->g.ns,
                                   rord ? h->pos_pl : nullptr, rord);
        done = true;
      }
    }
    if (!done)
      tr::launch_gemm_oct<T>(LevelBuf<T>::Bh(D, adj), D.sym_ldb, u, y, D.om, (int)h->g.S, st, bias,
                             scale_sn ? h->sig_s : nullptr, h->g.ns, rord ? h->pos_pl : nullptr, rord);
    tend(h);
    return;
  }
  if (!D.Kf) {
    do_gemm<T>(h, LevelBuf<T>::G(D, adj), u, y, D.A, st, scale_sn, bias, rord, comp);
    return;
  }
  T *tmp = LevelBuf<T>::fact(h);
  const int S = (int)h->g.S;
  tbegin(h, comp);
  gemm<T>(h, LevelBuf<T>::Lf(D, adj), u, tmp, D.Kf, S, D.A, st);
  gemm<T>(h, LevelBuf<T>::Rf(D, adj), tmp, y, D.A, S, D.Kf, st, bias, scale_sn ? h->sig_s : nullptr, h->g.ns,
          rord ? h->pos_pl : nullptr, rord);
  tend(h);
}

// Fig. lmg on level l >= 0 in ordinate form; f (level l's f buffer) is the
// right-hand side, the result is left in level l's u buffer.
template <typename T>
void mg_level(tr_handle *h, int l, bool adj, hipStream_t st);

template <typename Tc>
struct Coarse;

template <typename T>
void mg_level(tr_handle *h, int l, bool adj, hipStream_t st) {
  DevLevel &D = h->lv[l];
  const int nu_pre = h->prob.nu_pre;
  const int nu_post = l < h->top() && h->prob.nu_post_coarse > 0 ? h->prob.nu_post_coarse : h->prob.nu_post;
  T *f = LevelBuf<T>::f(D), *u = LevelBuf<T>::u(D);
  T *sa = LevelBuf<T>::sa(D), *sb = LevelBuf<T>::sb(D);
  DevLevel &Dc = h->lv[l - 1];
  // Forward: f holds the prepared right-hand side f~ = N^{-1} f, every
  // sweep reads one prepared vector (f~ itself, or f~ + sigma_s G u formed
  // by the GEMM epilogue) and the restricted residual is R sigma_s G du
  // (N commutes with the angular operators).  Adjoint: weak-form f, the
  // sweep forms f + sigma_s N s itself.
  // pre-smoothing (source iteration from zero)
  do_sweep<T>(h, l, f, nullptr, u, adj, st);
  T *s_prev = nullptr;
  for (int it = 1; it < nu_pre; ++it) {
    if (!adj) {
      level_scatter<T>(h, l, adj, u, sa, st, true, f, LevelBuf<T>::pin(D));
      do_sweep<T>(h, l, sa, nullptr, u, adj, st);
    } else {
      level_scatter<T>(h, l, adj, u, sa, st);
      do_sweep<T>(h, l, f, sa, u, adj, st);
    }
    s_prev = sa;
    std::swap(sa, sb);
  }
  // residual S (u - u_prev), restricted to level l-1 (forward: both terms
  // carry the same f~, which cancels)
  if (!adj)
    level_scatter<T>(h, l, adj, u, sa, st, true, s_prev ? f : nullptr);
  else
    level_scatter<T>(h, l, adj, u, sa, st);
  tbegin(h, C_TRANSFER);
  if (l - 1 == 0)
    tr::launch_restrict<T, double>(sa, s_prev, Dc.f64, adj ? D.Ra : D.Ru, D.first_child, D.n_child, Dc.P, h->sig_s,
                                   adj, h->g, st);
  else
    tr::launch_restrict<T, T>(sa, s_prev, LevelBuf<T>::f(Dc), adj ? D.Ra : D.Ru, D.first_child, D.n_child, Dc.P,
                              h->sig_s, adj, h->g, st, !adj && LevelBuf<T>::pin(Dc) ? h->pos_pl : nullptr, Dc.ord);
  tend(h);
  if (l - 1 == 0)
    do_coarse(h, Dc.f64, Dc.u64, h->prob.nu_coarse, adj, st);
  else
    mg_level<T>(h, l - 1, adj, st);
  tbegin(h, C_TRANSFER);
  if (l - 1 == 0)
    tr::launch_prolong<double, T>(Dc.u64, u, adj ? D.Pa : D.Pu, D.first_child, D.n_child, Dc.P, h->g.S, true, st);
  else
    tr::launch_prolong<T, T>(LevelBuf<T>::u(Dc), u, adj ? D.Pa : D.Pu, D.first_child, D.n_child, Dc.P, h->g.S, true,
                             st);
  tend(h);
  for (int it = 0; it < nu_post; ++it) {
    if (!adj) {
      level_scatter<T>(h, l, adj, u, sa, st, true, f, LevelBuf<T>::pin(D));
      do_sweep<T>(h, l, sa, nullptr, u, adj, st);
    } else {
      level_scatter<T>(h, l, adj, u, sa, st);
      do_sweep<T>(h, l, f, sa, u, adj, st);
    }
  }
}

// z = M^{-1} r (canonical FP64 in and out)
// Right-hand side of a preconditioner or sweep call in ordinate form:
// prepared (N^{-1} applied) for the forward direction, weak form for the
// adjoint.
template <typename Tin, typename Tout>
void convert_in(tr_handle *h, int level, bool adj, const Tin *r, Tout *f, hipStream_t st, double scale = 1.0) {
  DevLevel &D = h->lv[level];
  if (adj)
    tr::launch_convert<Tin, Tout>(r, f, D.P, h->g.S, nullptr, nullptr, st, scale);
  else
    tr::launch_convert_minv<Tin, Tout>(r, f, D.P, h->g, nullptr, D.winv, st, LevelBuf<Tout>::pin(D) ? h->pos_pl : nullptr, D.ord,
                                       scale);
}

// z = out_scale M^{-1} (in_scale r).  The scales keep the FP32 V-cycle's
// input at unit size whatever the scale of r (GMRES passes its unnormalised
// basis vectors with the normalising factor).  With z32 (FP32 preconditioner
// modes only) the result is also left in FP32 in z32 and z, if not null,
// is its exact FP64 image, so the flexible GMRES update can use the stored
// FP32 vectors.
void precondition(tr_handle *h, int mode, bool adj, const double *r, double *z, hipStream_t st,
                  double in_scale = 1.0, double out_scale = 1.0, float *z32 = nullptr) {
  const int L = h->top();
  h->n_precond++;
  DevLevel &D = h->lv[L];
  const double *pre_out = adj ? D.winv : nullptr, *post_out = nullptr;
  const bool mixed = (mode == TR_PREC_MIXED || mode == TR_PREC_MIXED_BF16) && L > 0;
  if (z32 && !mixed) throw std::runtime_error("internal: FP32 preconditioned vectors need an FP32 V-cycle");
  if (!z && !z32) throw std::runtime_error("internal: preconditioner without an output");
  if (mode == TR_PREC_SG || L == 0) {
    tbegin(h, C_OTHER);
    convert_in<double, double>(h, L, adj, r, D.f64, st, in_scale);
    tend(h);
    if (mode == TR_PREC_SG)
      do_sweep<double>(h, L, D.f64, nullptr, D.u64, adj, st);
    else
      do_coarse(h, D.f64, D.u64, h->prob.nu_coarse, adj, st);
    tbegin(h, C_OTHER);
    tr::launch_convert<double, double>(D.u64, z, D.P, h->g.S, pre_out, post_out, st, out_scale);
    tend(h);
    return;
  }
  if (mixed) {
    ensure_mixed(h);
    struct Split {  // FP32 scatter products for this V-cycle only
      tr_handle *h;
      ~Split() { h->split32 = false; }
    } split_guard{h};
    h->split32 = mode == TR_PREC_MIXED_BF16;
    tbegin(h, C_OTHER);
    convert_in<double, float>(h, L, adj, r, D.f32, st, in_scale);
    tend(h);
    mg_level<float>(h, L, adj, st);
    tbegin(h, C_OTHER);
    if (z32) {
      // the FP32 vector kept for the flexible update and (z) its FP64 copy
      // for the operator, in one pass
      tr::launch_convert<float, float>(D.u32, z32, D.P, h->g.S, pre_out, post_out, st, out_scale, z);
    } else {
      tr::launch_convert<float, double>(D.u32, z, D.P, h->g.S, pre_out, post_out, st, out_scale);
    }
    tend(h);
  } else {
    tbegin(h, C_OTHER);
    convert_in<double, double>(h, L, adj, r, D.f64, st, in_scale);
    tend(h);
    mg_level<double>(h, L, adj, st);
    tbegin(h, C_OTHER);
    tr::launch_convert<double, double>(D.u64, z, D.P, h->g.S, pre_out, post_out, st, out_scale);
    tend(h);
  }
}

// t = S~ x with the problem's scatter order (canonical FP64, finest level)
void outer_scatter(tr_handle *h, const double *x, double *t, hipStream_t st) {
  DevLevel &D = h->lv[h->top()];
  if (h->Bouter)
    tr::launch_gemm_oct<double>(h->Bouter, h->outer_ldb, x, t, h->outer_om, (int)h->g.S, st);
  else
    tr::launch_gemm<double>(h->Souter, x, t, D.A, (int)h->g.S, D.A, st);
}

// y = A x (adj: A^T x), canonical FP64 on the finest level
void apply_A(tr_handle *h, bool adj, const double *x, double *y, hipStream_t st) {
  DevLevel &D = h->lv[h->top()];
  tbegin(h, C_SCATTER_OUTER);
  outer_scatter(h, x, h->tmp, st);
  tend(h);
  tbegin(h, C_APPLY);
  tr::launch_apply(x, h->tmp, y, h->sig_t, h->sig_s, D.ord, D.w, D.P, h->g, adj, st);
  tend(h);
}

// y = A x for x held twice, in FP64 (x) and as the FP32 values it widens
// exactly (x32): the scatter product reads x, the transport stencil the
// half-size x32
void apply_A_pair(tr_handle *h, bool adj, const double *x, const float *x32, double *y, hipStream_t st) {
  DevLevel &D = h->lv[h->top()];
  tbegin(h, C_SCATTER_OUTER);
  outer_scatter(h, x, h->tmp, st);
  tend(h);
  tbegin(h, C_APPLY);
  tr::launch_apply(x32, h->tmp, y, h->sig_t, h->sig_s, D.ord, D.w, D.P, h->g, adj, st);
  tend(h);
}

double dot(tr_handle *h, const double *x, const double *y, long long n, hipStream_t st) {
  tr::launch_dot_partial(x, y, n, h->dot_partial, h->dot_blocks, st);
  tr::launch_dot_final(h->dot_partial, h->dot_blocks, h->dot_out, st);
  double v = 0;
  HIPCHK(hipMemcpyAsync(&v, h->dot_out, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return v;
}

bool mixed_mode(int mode) { return mode == TR_PREC_MIXED || mode == TR_PREC_MIXED_BF16; }

// Krylov workspace for GMRES(m): the basis V (m + 1 FP64 vectors), the work
// vector, and the preconditioned vectors Z of the flexible form when they
// are kept (FP64 for the FP64 preconditioners, FP32 for the FP32 ones).
// Returns 0 (recompute M^{-1}(V y) at each restart), 64 or 32.
int ensure_krylov(tr_handle *h, int m, int mode, int z_store) {
  const long long n = h->vec_len(h->top());
  while ((int)h->V.size() < m + 1) h->V.push_back(h->alloc<double>(n));
  if (!h->kw) h->kw = h->alloc<double>(n);
  if (!h->mdot_partial) h->mdot_partial = h->alloc<double>(32LL * h->dot_blocks);
  if (h->mdot_len < 2 * m + 4) {
    h->mdot_len = 2 * m + 4;
    h->mdot_out = h->alloc<double>(h->mdot_len);
  }
  h->kry_m = std::max(h->kry_m, m);
  if (z_store == TR_Z_RECOMPUTE) return 0;
  if (mixed_mode(mode) && h->top() > 0) {
    // a non-linear (FP32) preconditioner needs the flexible form: always
    // keep its vectors, in FP32
    try {
      while ((int)h->Z32.size() < m) h->Z32.push_back(h->alloc<float>(n));
    } catch (const std::bad_alloc &) {
      throw std::runtime_error("out of device memory for the FP32 preconditioned vectors of the flexible GMRES (" +
                               std::to_string((double)m * n * 4 / 1e9) +
                               " GB); z_store = TR_Z_RECOMPUTE runs without them");
    }
    return 32;
  }
  if ((int)h->Z.size() >= m) return 64;
  const size_t need = (size_t)(m - h->Z.size()) * n * sizeof(double);
  if (z_store == TR_Z_AUTO) {
    // a linear (FP64) preconditioner gives the same iterates either way:
    // keep the vectors when they fit in half of the free memory
    size_t fr = 0, tot = 0;
    if (!h->dry) HIPCHK(hipMemGetInfo(&fr, &tot));
    if (h->dry || need >= fr / 2) return 0;
  }
  while ((int)h->Z.size() < m) h->Z.push_back(h->alloc<double>(n));
  return 64;
}

// One Arnoldi orthogonalisation in two passes over the basis (modified
// Gram-Schmidt in its inverse compact WY form, Swirydowicz et al. 2020):
//   pass 1: s_i = v_i . w (i <= j) and the new Gram row l_i = v_j . v_i (i < j)
//   host:   h = (I + L)^{-1} s, L strictly lower with the Gram rows, which
//           reproduces the sequential projections of modified Gram-Schmidt
//   pass 2: w -= sum_i h_i v_i, returning |w|^2.
// The basis is stored unnormalised: v_i = vs[i] V[i]; the scales enter the
// host arithmetic only.  Lg holds the Gram rows (row j written here); hcol
// receives h; returns |w|^2 after the update.
double arnoldi_orth(tr_handle *h, int j, double *W, const std::vector<double> &vs, std::vector<double> &Lg, int m,
                    double *hcol, long long n, hipStream_t st) {
  const int k = j + 1;
  std::vector<const double *> X(h->V.begin(), h->V.begin() + k);
  int off = 0;
  std::vector<std::array<int, 3>> chunks;  // q0, c, kz
  for (int q0 = 0; q0 < k; q0 += 16) {
    const int c = std::min(16, k - q0);
    const int kz = std::min(c, std::max(0, j - q0));
    tr::launch_multi_dot(n, c, X.data() + q0, W, kz, h->V[j], h->mdot_partial, h->dot_blocks, h->mdot_out + off,
                         st);
    chunks.push_back({q0, c, kz});
    off += c + kz;
  }
  std::vector<double> r(off);
  HIPCHK(hipMemcpyAsync(r.data(), h->mdot_out, off * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<double> sv(k);
  off = 0;
  for (auto &ch : chunks) {
    for (int q = 0; q < ch[1]; ++q) sv[ch[0] + q] = vs[ch[0] + q] * r[off + q];
    for (int q = 0; q < ch[2]; ++q) Lg[(size_t)j * m + ch[0] + q] = vs[j] * vs[ch[0] + q] * r[off + ch[1] + q];
    off += ch[1] + ch[2];
  }
  std::vector<double> c(k);
  for (int i = 0; i < k; ++i) {
    double t = sv[i];
    for (int q = 0; q < i; ++q) t -= Lg[(size_t)i * m + q] * hcol[q];
    hcol[i] = t;
    c[i] = -t * vs[i];
  }
  tr::launch_multi_axpy_norm(n, k, X.data(), c.data(), W, h->dot_partial, h->dot_blocks, h->dot_out, st);
  double nrm2 = 0;
  HIPCHK(hipMemcpyAsync(&nrm2, h->dot_out, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return nrm2;
}

// Restarted right-preconditioned GMRES(m), x0 = 0, modified Gram-Schmidt.
// The Krylov basis is kept unnormalised with host-side scales (saves a
// normalisation pass per step): the next basis vector is the updated work
// vector itself, whose buffer changes place with the work buffer.  The
// preconditioner always receives the unit basis vector v_j (its scale is
// applied in the input conversion).  With the preconditioned vectors kept
// this is flexible GMRES (x += sum y_i z_i); without them x += M^{-1} V y.
int gmres(tr_handle *h, bool adj, const double *b, double *x, const tr_solve_opts *o, tr_solve_stats *stats,
          hipStream_t st) {
  const int m = o->restart;
  const int zkind = ensure_krylov(h, m, o->prec_mode, o->z_store);
  const long long n = h->vec_len(h->top());
  tr::launch_fill<double>(x, n, 0.0, st);
  tbegin(h, C_ORTH);
  const double bnorm = std::sqrt(dot(h, b, b, n, st));
  tend(h);
  stats->iters = 0;
  stats->restarts = 0;
  stats->converged = 0;
  stats->rel_res = 0;
  stats->flexible = zkind;
  if (bnorm == 0.0) {
    stats->converged = 1;
    return TR_OK;
  }
  HIPCHK(hipMemcpyAsync(h->V[0], b, n * sizeof(double), hipMemcpyDeviceToDevice, st));  // r0 = b
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m), Lg((size_t)m * m), hcol(m + 1),
      vs(m + 1), yc(m);
  for (int cycle = 0; cycle <= o->max_restarts; ++cycle) {
    tbegin(h, C_ORTH);
    const double beta = std::sqrt(dot(h, h->V[0], h->V[0], n, st));
    tend(h);
    stats->rel_res = beta / bnorm;
    stats->restarts = cycle;
    if (beta / bnorm < o->tol) {
      stats->converged = 1;
      return TR_OK;
    }
    if (cycle == o->max_restarts) break;
    vs[0] = 1.0 / beta;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      // z_j = M^{-1} v_j (v_j = vs[j] V[j]), w = A z_j
      double *zj = zkind == 64 ? h->Z[j] : h->tmp2;
      double *W = h->kw;
      precondition(h, o->prec_mode, adj, h->V[j], zj, st, vs[j], 1.0, zkind == 32 ? h->Z32[j] : nullptr);
      if (zkind == 32)
        apply_A_pair(h, adj, zj, h->Z32[j], W, st);  // the stencil reads the FP32 copy
      else
        apply_A(h, adj, zj, W, st);
      stats->iters++;
      // modified Gram-Schmidt (two passes over the basis, see arnoldi_orth)
      tbegin(h, C_ORTH);
      const double hn = std::sqrt(arnoldi_orth(h, j, W, vs, Lg, m, hcol.data(), n, st));
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hcol[i];
      tend(h);
      H[(size_t)(j + 1) * m + j] = hn;
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = t;
      }
      const double rho = std::hypot(H[(size_t)j * m + j], hn);
      cs[j] = H[(size_t)j * m + j] / rho;
      sn[j] = hn / rho;
      const bool breakdown = hn == 0.0;
      if (!breakdown) {
        // v_{j+1} = W / hn: W becomes V[j+1]
        std::swap(h->V[j + 1], h->kw);
        vs[j + 1] = 1.0 / hn;
      }
      H[(size_t)j * m + j] = rho;
      H[(size_t)(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      k = j + 1;
      if (std::fabs(gv[j + 1]) / bnorm < o->tol || breakdown) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double t = gv[i];
      for (int jj = i + 1; jj < k; ++jj) t -= H[(size_t)i * m + jj] * y[jj];
      y[i] = t / H[(size_t)i * m + i];
    }
    double *w = h->kw;
    tbegin(h, C_ORTH);
    if (zkind == 64) {
      tr::launch_multi_axpy(n, k, h->Z.data(), y.data(), x, st);
    } else if (zkind == 32) {
      tr::launch_multi_axpy_f32(n, k, h->Z32.data(), y.data(), x, st);
    } else {
      for (int i = 0; i < k; ++i) yc[i] = y[i] * vs[i];
      tr::launch_fill<double>(w, n, 0.0, st);
      tr::launch_multi_axpy(n, k, h->V.data(), yc.data(), w, st);
    }
    tend(h);
    if (!zkind) {
      // x += M^{-1}(V y), the preconditioner's input scaled to about unit
      // size (|V y| = |y| for the orthonormal basis)
      double ny = 0;
      for (int i = 0; i < k; ++i) ny += y[i] * y[i];
      ny = std::sqrt(ny);
      if (ny > 0) {
        precondition(h, o->prec_mode, adj, w, h->tmp2, st, 1.0 / ny, ny);
        tbegin(h, C_ORTH);
        tr::launch_axpy(n, 1.0, h->tmp2, x, st);
        tend(h);
      }
    }
    // explicit residual r = b - A x into V[0]
    apply_A(h, adj, x, w, st);
    tbegin(h, C_ORTH);
    tr::launch_axpby(n, 1.0, b, -1.0, w, h->V[0], st);
    tend(h);
  }
  return TR_ERR_NOCONV;
}

// Right-preconditioned BiCGStab (the paper's Krylov method, Section 3) from
// x = 0, van der Vorst's recurrences: per iteration two preconditioner
// applications and two operator applications.  When the recurrence residual
// falls below tol |b| the explicit residual b - A x decides; a failed test
// restarts the recurrences from it.  Iteration limit: restart x (max_restarts
// + 1), the GMRES budget.  FP32 preconditioners receive unit-norm inputs.
int bicgstab(tr_handle *h, bool adj, const double *b, double *x, const tr_solve_opts *o, tr_solve_stats *stats,
             hipStream_t st) {
  ensure_krylov(h, 7, TR_PREC_F64, TR_Z_RECOMPUTE);
  const long long n = h->vec_len(h->top());
  double *r = h->V[0], *rhat = h->V[1], *p = h->V[2], *v = h->V[3], *s = h->V[4], *t = h->V[5], *ph = h->V[6],
         *sh = h->V[7];
  const bool mixed = mixed_mode(o->prec_mode);
  const long long max_iters = (long long)o->restart * (o->max_restarts + 1);
  tr::launch_fill<double>(x, n, 0.0, st);
  tbegin(h, C_ORTH);
  const double bnorm = std::sqrt(dot(h, b, b, n, st));
  tend(h);
  stats->iters = stats->restarts = stats->converged = 0;
  stats->rel_res = 0;
  stats->flexible = 0;
  if (bnorm == 0.0) {
    stats->converged = 1;
    return TR_OK;
  }
  auto prec = [&](const double *in, double *out) {
    double sc = 1.0;
    if (mixed) {
      const double nn = std::sqrt(dot(h, in, in, n, st));
      if (nn > 0) sc = 1.0 / nn;
    }
    precondition(h, o->prec_mode, adj, in, out, st, sc, 1.0 / sc);
  };
  HIPCHK(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  long long iters = 0;
  while (iters < max_iters) {
    HIPCHK(hipMemcpyAsync(rhat, r, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    tr::launch_fill<double>(p, n, 0.0, st);
    tr::launch_fill<double>(v, n, 0.0, st);
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    while (iters < max_iters) {
      tbegin(h, C_ORTH);
      const double rho = dot(h, rhat, r, n, st);
      tend(h);
      if (rho == 0.0) break;
      const double beta = (rho / rho_prev) * (alpha / omega);
      tbegin(h, C_ORTH);
      tr::launch_scal(n, beta, p, st);  // p = r + beta (p - omega v)
      {
        const double *xs[2] = {r, v};
        const double cs2[2] = {1.0, -beta * omega};
        tr::launch_multi_axpy(n, 2, xs, cs2, p, st);
      }
      tend(h);
      prec(p, ph);
      apply_A(h, adj, ph, v, st);
      tbegin(h, C_ORTH);
      alpha = rho / dot(h, rhat, v, n, st);
      tr::launch_axpby(n, 1.0, r, -alpha, v, s, st);
      const double sn = std::sqrt(dot(h, s, s, n, st));
      tend(h);
      ++iters;
      if (sn / bnorm < o->tol) {
        tbegin(h, C_ORTH);
        tr::launch_axpy(n, alpha, ph, x, st);
        tend(h);
        std::swap(h->V[0], h->V[4]);
        r = h->V[0];
        s = h->V[4];
        break;
      }
      prec(s, sh);
      apply_A(h, adj, sh, t, st);
      tbegin(h, C_ORTH);
      const double ts = dot(h, t, s, n, st), tt = dot(h, t, t, n, st);
      omega = tt > 0 ? ts / tt : 0.0;
      {
        const double *xs[2] = {ph, sh};
        const double cs2[2] = {alpha, omega};
        tr::launch_multi_axpy(n, 2, xs, cs2, x, st);
      }
      tr::launch_axpby(n, 1.0, s, -omega, t, r, st);
      const double rn = std::sqrt(dot(h, r, r, n, st));
      tend(h);
      rho_prev = rho;
      if (rn / bnorm < o->tol || omega == 0.0) break;
    }
    // acceptance by the explicit residual r = b - A x
    apply_A(h, adj, x, t, st);
    tbegin(h, C_ORTH);
    tr::launch_axpby(n, 1.0, b, -1.0, t, r, st);
    const double rel = std::sqrt(dot(h, r, r, n, st)) / bnorm;
    tend(h);
    stats->iters = (int)iters;
    stats->rel_res = rel;
    if (rel < o->tol) {
      stats->converged = 1;
      return TR_OK;
    }
    stats->restarts++;
  }
  return TR_ERR_NOCONV;
}

void fill_stats(tr_handle *h, tr_solve_stats *s, double ms_total) {
  s->ms_total = ms_total;
  s->n_precond = (int)h->n_precond;
  s->sweep_dof_updates = h->sweep_dofs;
  s->coarse_steps = h->coarse_steps;
  s->ms_sweep = s->ms_scatter = s->ms_transfer = s->ms_coarse = s->ms_apply = s->ms_orth = s->ms_other = 0;
  s->n_sweep = s->n_scatter = s->n_coarse = 0;
  s->ms_sweep_finest = 0;
  s->n_sweep_finest = 0;
  s->ms_scatter_outer = 0;
  s->n_scatter_outer = 0;
  s->ms_scatter_finest = 0;
  s->n_scatter_finest = 0;
  if (!h->timer) return;
  for (auto &r : h->timer->recs) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    switch (r.comp) {
      case C_SWEEP: s->ms_sweep += ms; s->n_sweep++; break;
      case C_SWEEP_FINE: s->ms_sweep += ms; s->n_sweep++; s->ms_sweep_finest += ms; s->n_sweep_finest++; break;
      case C_SCATTER: s->ms_scatter += ms; s->n_scatter++; break;
      case C_SCATTER_OUTER:
        s->ms_scatter += ms; s->n_scatter++; s->ms_scatter_outer += ms; s->n_scatter_outer++;
        break;
      case C_SCATTER_FINE:
        s->ms_scatter += ms; s->n_scatter++; s->ms_scatter_finest += ms; s->n_scatter_finest++;
        break;
      case C_TRANSFER: s->ms_transfer += ms; break;
      case C_COARSE: s->ms_coarse += ms; s->n_coarse++; break;
      case C_APPLY: s->ms_apply += ms; break;
      case C_ORTH: s->ms_orth += ms; break;
      default: s->ms_other += ms; break;
    }
  }
}

int translate(const std::function<int()> &fn) {
  try {
    return fn();
  } catch (const ArgError &e) {
    return fail(TR_ERR_ARG, e.msg);
  } catch (const HipError &e) {
    return fail(TR_ERR_HIP, std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
  } catch (const std::bad_alloc &) {
    return fail(TR_ERR_ALLOC, "out of memory");
  } catch (const std::exception &e) {
    return fail(TR_ERR_HIP, e.what());
  }
}

// Device vectors are read and written with 16-byte accesses.
bool misaligned(const void *p) { return p && ((uintptr_t)p & 15) != 0; }
template <typename... P>
bool any_misaligned(P... p) {
  return (misaligned(p) || ...);
}
#define TR_CHECK_ALIGNED(...) \
  if (any_misaligned(__VA_ARGS__)) return fail(TR_ERR_ARG, "device buffers must be 16-byte aligned")

bool valid_mode(int m) {
  return m == TR_PREC_F64 || m == TR_PREC_MIXED || m == TR_PREC_SG || m == TR_PREC_MIXED_BF16;
}
bool valid_zstore(int z) { return z == TR_Z_AUTO || z == TR_Z_KEEP || z == TR_Z_RECOMPUTE; }

int check_level(tr_handle *h, int level) {
  if (!h) return fail(TR_ERR_ARG, "null handle");
  if (level < 0 || level > h->top()) return fail(TR_ERR_ARG, "level out of range");
  return TR_OK;
}

hipStream_t S(tr_stream s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

// ------------------------------------------------- allocation-free coarse solve
// Scratch of tr_coarse_gs_noalloc: word 0 is the wait-timeout error word,
// the update counters start at word 64 (256 bytes).  One copy per device,
// held until the process ends; every call on a device shares it.
constexpr long long kScratchCounters = 1LL << 20;
constexpr long long kScratchHeader = 64;
static __device__ __align__(256) unsigned scratch[kScratchHeader + kScratchCounters];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (resolved once per device, with
// that device current; host code never uses the array's own name).
unsigned *scratch_ptr() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw std::runtime_error("device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw std::runtime_error("no device address for the coarse-solve scratch");
    g_scratch_ptr[dev] = static_cast<unsigned *>(p);
  }
  return g_scratch_ptr[dev];
}

// =================================================================== ABI
extern "C" {

const char *tr_last_error(void) { return g_err.c_str(); }

int tr_setup(const tr_problem *prob, tr_handle **out) {
  if (!prob || !out) return fail(TR_ERR_ARG, "null argument");
  *out = nullptr;
  tr_handle *h = nullptr;
  int rc = translate([&]() {
    h = new tr_handle();
    // TR_COARSE_GS=barrier (barrier_fence: with cache maintenance fences)
    // selects the step-synchronous coarse solve, TR_COARSE_GS=cell the
    // dataflow form per cell, for comparison; the default is the dataflow
    // form per brick where the grid allows it, else per cell
    const char *gs = std::getenv("TR_COARSE_GS");
    h->gs_flow = !(gs && std::strncmp(gs, "barrier", 7) == 0);
    h->gs_coh = !(gs && std::strcmp(gs, "barrier_fence") == 0);
    h->gs_brick = !(gs && std::strcmp(gs, "cell") == 0);
    build(h, prob);
    scratch_ptr();  // the allocation-free coarse solve's scratch on this device
    return TR_OK;
  });
  if (rc != TR_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return TR_OK;
}

void tr_destroy(tr_handle *h) { delete h; }

int tr_info(const tr_handle *h, tr_info_t *out) {
  if (!h || !out) return fail(TR_ERR_ARG, "null argument");
  std::memset(out, 0, sizeof *out);
  out->dim = h->g.dim;
  out->cells = (int)h->g.C;
  out->spatial_dofs = (int)h->g.S;
  out->n_levels = (int)h->lv.size();
  for (size_t l = 0; l < h->lv.size(); ++l) out->patches[l] = h->lv[l].P;
  out->order_outer = h->prob.order;
  out->device_bytes = h->bytes;
  for (size_t l = 0; l < h->lv.size(); ++l) {
    const DevLevel &D = h->lv[l];
    out->scatter_form[l] = D.symR ? TR_SCATTER_OCTANT : D.Kf ? TR_SCATTER_FACTORED : TR_SCATTER_DENSE;
    out->scatter_axes[l] = D.symR;
    out->scatter_k[l] = D.Kf;
  }
  out->outer_axes = h->Bouter ? h->outer_R : 0;
  out->sweep_lds[0] = tr::sweep_lds_fits<double>(h->pl, h->g, false) ? 1 : 0;
  out->sweep_lds[1] = tr::sweep_lds_fits<float>(h->pl, h->g, false) ? 1 : 0;
  out->sweep_pair[0] = h->bpl.nplanes > 0 && tr::sweep_pair_fits<double>(h->bpl) ? 1 : 0;
  out->sweep_pair[1] = h->bpl.nplanes > 0 && tr::sweep_pair_fits<float>(h->bpl) ? 1 : 0;
  return TR_OK;
}

int tr_set_sigma(tr_handle *h, const double *sigma_t, const double *sigma_s, tr_stream st) {
  if (!h || !sigma_t || !sigma_s) return fail(TR_ERR_ARG, "null argument");
  return translate([&]() {
    // the same checks as tr_setup, on a host copy; the handle keeps its
    // cross sections when they fail
    std::vector<double> t(h->g.C), sc(h->g.C);
    HIPCHK(hipMemcpyAsync(t.data(), sigma_t, h->g.C * sizeof(double), hipMemcpyDeviceToHost, S(st)));
    HIPCHK(hipMemcpyAsync(sc.data(), sigma_s, h->g.C * sizeof(double), hipMemcpyDeviceToHost, S(st)));
    HIPCHK(hipStreamSynchronize(S(st)));
    for (long long j = 0; j < h->g.C; ++j) {
      if (!(std::isfinite(t[j]) && t[j] > 0)) throw ArgError{"sigma_t must be finite and > 0 (cell " + std::to_string(j) + ")"};
      if (!(std::isfinite(sc[j]) && sc[j] >= 0))
        throw ArgError{"sigma_s must be finite and >= 0 (cell " + std::to_string(j) + ")"};
    }
    HIPCHK(hipMemcpyAsync(h->sig_t, sigma_t, h->g.C * sizeof(double), hipMemcpyDeviceToDevice, S(st)));
    HIPCHK(hipMemcpyAsync(h->sig_s, sigma_s, h->g.C * sizeof(double), hipMemcpyDeviceToDevice, S(st)));
    tr::launch_sigma_planes(h->sig_t, h->sig_s, h->pl, h->g, h->sig_pl, S(st));
    if (h->d_slots) tr::launch_sigma_planes(h->sig_t, h->sig_s, slot_planes(h), h->g, h->sig_pb, S(st));
    h->sig_t_host = t;
    h->sig_s_host = sc;
    return TR_OK;
  });
}

int tr_response(tr_handle *h, const double *w, const double *phi, double *R, tr_stream st) {
  if (!h || !w || !phi || !R) return fail(TR_ERR_ARG, "null argument");
  TR_CHECK_ALIGNED(w, phi);
  return translate([&]() {
    *R = dot(h, w, phi, h->vec_len(h->top()), S(st));
    return TR_OK;
  });
}

int tr_workspace_bytes(const tr_problem *prob, const tr_solve_opts *o, size_t *bytes) {
  if (!prob || !bytes) return fail(TR_ERR_ARG, "null argument");
  *bytes = 0;
  if (o && (o->restart < 1 || o->restart > 200 || !valid_mode(o->prec_mode) || !valid_zstore(o->z_store)))
    return fail(TR_ERR_ARG, "bad solver options");
  std::unique_ptr<tr_handle> h(new tr_handle());
  h->dry = true;
  return translate([&]() {
    build(h.get(), prob);
    if (o) {
      // what a solve with these options adds: the FP32 level buffers, the
      // Krylov workspace, the split-BF16 level matrices, the coarse solve's
      // schedule and counters
      const bool mixed = mixed_mode(o->prec_mode) && h->top() > 0;
      if (mixed) ensure_mixed(h.get());
      ensure_krylov(h.get(), o->restart, o->prec_mode, o->z_store == TR_Z_AUTO ? TR_Z_KEEP : o->z_store);
      if (o->prec_mode == TR_PREC_MIXED_BF16 && mixed)
        for (int l = 1; l <= h->top(); ++l) {
          DevLevel &D = h->lv[l];
          if (D.symR) {
            split_blocks(h.get(), D, D.Bh32, nullptr);
          } else if (D.Kf) {
            split_of(h.get(), D.Rt32, D.Kf, D.A, nullptr);
            split_of(h.get(), D.L32, D.A, D.Kf, nullptr);
          } else {
            split_of(h.get(), D.G32, D.A, D.A, nullptr);
          }
        }
      if (o->prec_mode != TR_PREC_SG) {
        gs_schedule(h.get(), h->prob.nu_coarse, false);
        ensure_coarse_buffers(h.get());
      }
    }
    *bytes = h->bytes;
    return TR_OK;
  });
}

int tr_rhs(tr_handle *h, const double *q_cell, const tr_inflow *in, double *b, tr_stream st) {
  if (!h || !b) return fail(TR_ERR_ARG, "null argument");
  TR_CHECK_ALIGNED(b);
  return translate([&]() {
    const int L = h->top();
    DevLevel &D = h->lv[L];
    const tr::HostLevel &H = h->ang.lv[L];
    const Grid &g = h->g;
    tr::launch_rhs_volume(b, q_cell, D.ipsi, D.A, g, S(st));
    if (!in || in->kind == TR_INFLOW_NONE) return TR_OK;
    if (in->kind != TR_INFLOW_ISO && in->kind != TR_INFLOW_BEAM) throw ArgError{"unknown inflow kind"};
    if (in->axis < 0 || in->axis >= g.dim || (in->side != 0 && in->side != 1)) throw ArgError{"bad inflow face"};
    const int ax = in->axis, side = in->side;
    const double sigma_f = side == 0 ? -1.0 : 1.0;
    // cells of the face box
    std::vector<int> cells;
    for (int iz = 0; iz < g.n[2]; ++iz)
      for (int iy = 0; iy < g.n[1]; ++iy)
        for (int ix = 0; ix < g.n[0]; ++ix) {
          int c[3] = {ix, iy, iz};
          if (c[ax] != (side == 0 ? 0 : g.n[ax] - 1)) continue;
          bool ok = true;
          for (int d = 0; d < g.dim; ++d)
            if (d != ax && (c[d] < in->lo[d] || c[d] > in->hi[d])) ok = false;
          if (ok) cells.push_back(ix + g.n[0] * (iy + g.n[1] * iz));
        }
    // face integral of each node: nodes on the face get prod_{other} h / 2
    std::vector<double> fint(g.ns, 0.0);
    for (int b2 = 0; b2 < g.ns; ++b2) {
      if (((b2 >> ax) & 1) != side) continue;
      double v = 1.0;
      for (int d = 0; d < g.dim; ++d)
        if (d != ax) v *= g.h[d] / 2.0;
      fint[b2] = v;
    }
    std::vector<double> coef(D.A, 0.0);
    if (in->kind == TR_INFLOW_ISO) {
      for (int q = 0; q < D.P; ++q) {
        const double s = (H.octant[q] >> ax) & 1 ? -1.0 : 1.0;
        if (sigma_f * s >= 0) continue;  // not incoming through this face
        for (int m = 0; m < 3; ++m) coef[3 * q + m] = -sigma_f * in->value * H.iom[3 * (3 * q + m) + ax];
      }
    } else {
      double dn = std::sqrt(in->direction[0] * in->direction[0] + in->direction[1] * in->direction[1] +
                            in->direction[2] * in->direction[2]);
      if (!(dn > 0)) throw ArgError{"beam direction must be nonzero"};
      tr::V3 d{in->direction[0] / dn, in->direction[1] / dn, in->direction[2] / dn};
      const double dd[3] = {d.x, d.y, d.z};
      if (-sigma_f * dd[ax] <= 0) throw ArgError{"beam direction does not enter through the face"};
      std::vector<std::pair<int, std::array<double, 3>>> hits;
      for (int q = 0; q < D.P; ++q) {
        const tr::PatchNode &pn = h->ang.tree[H.node[q]];
        double sx = (pn.octant & 1) ? -1 : 1, sy = (pn.octant & 2) ? -1 : 1, sz = (pn.octant & 4) ? -1 : 1;
        if (sx * d.x + sy * d.y + sz * d.z <= 1e-14) continue;
        double psi[3];
        tr::lin_basis(pn, d, psi);
        if (psi[0] >= -1e-12 && psi[1] >= -1e-12 && psi[2] >= -1e-12) hits.push_back({q, {psi[0], psi[1], psi[2]}});
      }
      // Lin: the patch functions' values at the direction; Const: the
      // constant 1, a third in each of the three coincident ordinates
      for (auto &hq : hits)
        for (int m = 0; m < 3; ++m)
          coef[3 * hq.first + m] =
              in->value * (h->ang.const_basis ? 1.0 / 3.0 : hq.second[m]) / (double)hits.size();
    }
    TmpBuf tcoef(D.A * sizeof(double)), tcells(cells.size() * sizeof(int)), tfint(g.ns * sizeof(double));
    double *dcoef = tcoef.as<double>(), *dfint = tfint.as<double>();
    int *dcells = tcells.as<int>();
    HIPCHK(hipMemcpyAsync(dcoef, coef.data(), D.A * sizeof(double), hipMemcpyHostToDevice, S(st)));
    if (!cells.empty())
      HIPCHK(hipMemcpyAsync(dcells, cells.data(), cells.size() * sizeof(int), hipMemcpyHostToDevice, S(st)));
    HIPCHK(hipMemcpyAsync(dfint, fint.data(), g.ns * sizeof(double), hipMemcpyHostToDevice, S(st)));
    tr::launch_rhs_face(b, dcoef, dcells, (int)cells.size(), dfint, D.A, g, S(st));
    HIPCHK(hipStreamSynchronize(S(st)));
    return TR_OK;
  });
}

int tr_detector(tr_handle *h, const int lo[3], const int hi[3], double *w, tr_stream st) {
  if (!h || !lo || !hi || !w) return fail(TR_ERR_ARG, "null argument");
  TR_CHECK_ALIGNED(w);
  return translate([&]() {
    DevLevel &D = h->lv[h->top()];
    tr::launch_detector(w, D.ipsi, D.A, h->g, lo, hi, S(st));
    return TR_OK;
  });
}

static int sweep_common(tr_handle *h, int level, int prec, const void *g, void *phi, bool adj, tr_stream st) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!g || !phi) return fail(TR_ERR_ARG, "null buffer");
  TR_CHECK_ALIGNED(g, phi);
  if (prec != TR_F64 && prec != TR_F32) return fail(TR_ERR_ARG, "bad precision");
  return translate([&]() {
    DevLevel &D = h->lv[level];
    const double *pre_out = adj ? D.winv : nullptr;
    if (prec == TR_F64) {
      convert_in<double, double>(h, level, adj, (const double *)g, D.f64, S(st));
      do_sweep<double>(h, level, D.f64, nullptr, D.u64, adj, S(st));
      tr::launch_convert<double, double>(D.u64, (double *)phi, D.P, h->g.S, pre_out, nullptr, S(st));
    } else if (level > 0) {
      ensure_mixed(h);
      convert_in<float, float>(h, level, adj, (const float *)g, D.f32, S(st));
      do_sweep<float>(h, level, D.f32, nullptr, D.u32, adj, S(st));
      tr::launch_convert<float, float>(D.u32, (float *)phi, D.P, h->g.S, pre_out, nullptr, S(st));
    } else {
      // level 0 has no FP32 buffers: scratch for this call
      const size_t bytes = (size_t)h->vec_len(level) * sizeof(float);
      TmpBuf tf(bytes), tu(bytes);
      float *f = tf.as<float>(), *u = tu.as<float>();
      convert_in<float, float>(h, level, adj, (const float *)g, f, S(st));
      do_sweep<float>(h, level, f, nullptr, u, adj, S(st));
      tr::launch_convert<float, float>(u, (float *)phi, D.P, h->g.S, pre_out, nullptr, S(st));
      HIPCHK(hipStreamSynchronize(S(st)));
    }
    return TR_OK;
  });
}

int tr_sweep(tr_handle *h, int level, int prec, const void *g, void *phi, tr_stream st) {
  return sweep_common(h, level, prec, g, phi, false, st);
}

int tr_sweep_adjoint(tr_handle *h, int level, int prec, const void *g, void *lam, tr_stream st) {
  return sweep_common(h, level, prec, g, lam, true, st);
}

int tr_scatter(tr_handle *h, int level, int outer, int prec, const void *phi, void *s, tr_stream st) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!phi || !s) return fail(TR_ERR_ARG, "null buffer");
  TR_CHECK_ALIGNED(phi, s);
  if (outer && level != h->top()) return fail(TR_ERR_ARG, "the problem operator lives on the finest level");
  if (prec != TR_F64 && prec != TR_F32 && prec != TR_F32_SPLIT) return fail(TR_ERR_ARG, "bad precision");
  if (outer && prec != TR_F64) return fail(TR_ERR_UNSUPPORTED, "the problem operator is FP64 only");
  return translate([&]() {
    DevLevel &D = h->lv[level];
    const int Sn = (int)h->g.S;
    if (prec == TR_F64) {
      double *t = level == h->top() ? h->tmp : D.sa64;
      if (outer)
        outer_scatter(h, (const double *)phi, t, S(st));
      else if (D.symR)
        tr::launch_gemm_oct<double>(D.Bc64, D.sym_ldb, (const double *)phi, t, D.om, Sn, S(st));
      else
        tr::launch_gemm<double>(D.St64, (const double *)phi, t, D.A, Sn, D.A, S(st));
      tr::launch_scale_sn<double>(t, (double *)s, h->sig_s, D.A, h->g, S(st));
    } else {
      float *t = reinterpret_cast<float *>(D.sa64);  // the level's FP64 work buffer holds n floats
      if (prec == TR_F32_SPLIT && D.symR)
        tr::launch_gemm_oct_bf16x3(split_blocks(h, D, D.Bc32, S(st)), tr::split_rows_kp(D.sym_ldb),
                                   (const float *)phi, t, D.om, Sn, S(st));
      else if (prec == TR_F32_SPLIT)
        tr::launch_gemm_bf16x3(split_of(h, D.St32, D.A, D.A, S(st)), (const float *)phi, t, D.A, Sn, D.A, S(st));
      else if (D.symR)
        tr::launch_gemm_oct<float>(D.Bc32, D.sym_ldb, (const float *)phi, t, D.om, Sn, S(st));
      else
        tr::launch_gemm<float>(D.St32, (const float *)phi, t, D.A, Sn, D.A, S(st));
      tr::launch_scale_sn<float>(t, (float *)s, h->sig_s, D.A, h->g, S(st));
    }
    return TR_OK;
  });
}

int tr_apply(tr_handle *h, const double *x, double *y, tr_stream st) {
  if (!h || !x || !y) return fail(TR_ERR_ARG, "null argument");
  TR_CHECK_ALIGNED(x, y);
  return translate([&]() {
    apply_A(h, false, x, y, S(st));
    return TR_OK;
  });
}

int tr_transfer(tr_handle *h, int level, int dir, int prec, const void *in, void *out, tr_stream st) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (level < 1) return fail(TR_ERR_ARG, "transfers act between levels l-1 and l >= 1");
  if (!in || !out) return fail(TR_ERR_ARG, "null buffer");
  TR_CHECK_ALIGNED(in, out);
  if (dir != TR_RESTRICT && dir != TR_PROLONG) return fail(TR_ERR_ARG, "bad direction");
  return translate([&]() {
    DevLevel &D = h->lv[level], &Dc = h->lv[level - 1];
    if (dir == TR_PROLONG) {
      if (prec == TR_F64)
        tr::launch_prolong<double, double>((const double *)in, (double *)out, D.Pc, D.first_child, D.n_child,
                                           h->lv[level - 1].P, h->g.S, false, S(st));
      else
        tr::launch_prolong<float, float>((const float *)in, (float *)out, D.Pc, D.first_child, D.n_child,
                                         h->lv[level - 1].P, h->g.S, false, S(st));
    } else {
      if (prec == TR_F64)
        tr::launch_restrict<double, double>((const double *)in, nullptr, (double *)out, D.Rc, D.first_child,
                                            D.n_child, Dc.P, nullptr, false, h->g, S(st));
      else
        tr::launch_restrict<float, float>((const float *)in, nullptr, (float *)out, D.Rc, D.first_child, D.n_child,
                                          Dc.P, nullptr, false, h->g, S(st));
    }
    return TR_OK;
  });
}

int tr_coarse_gs(tr_handle *h, int nu, int adjoint, const double *f, double *phi, tr_stream st) {
  if (!h || !f || !phi) return fail(TR_ERR_ARG, "null argument");
  TR_CHECK_ALIGNED(f, phi);
  if (nu < 1) return fail(TR_ERR_ARG, "nu must be >= 1");
  return translate([&]() {
    DevLevel &D = h->lv[0];
    const bool adj = adjoint != 0;
    convert_in<double, double>(h, 0, adj, f, D.f64, S(st));
    do_coarse(h, D.f64, D.u64, nu, adj, S(st));
    tr::launch_convert<double, double>(D.u64, phi, D.P, h->g.S, adj ? D.winv : nullptr, nullptr, S(st));
    check_barrier(h, S(st));
    return TR_OK;
  });
}

int tr_coarse_gs_noalloc(tr_handle *h, int nu, int adjoint, const double *f, double *phi, tr_stream st) {
  if (!h || !f || !phi) return fail(TR_ERR_ARG, "null argument");
  TR_CHECK_ALIGNED(f, phi);
  if (nu < 1) return fail(TR_ERR_ARG, "nu must be >= 1");
  const bool adj = adjoint != 0;
  const tr_handle::GsSchedule *sc = nullptr;
  for (auto &e : h->gs_sched)
    if (e.nu == nu && e.adj == adj) sc = &e;
  if (!sc)
    return fail(TR_ERR_ARG, "no schedule for this sweep count: the problem's nu_coarse is prepared at setup, "
                            "other counts after one tr_coarse_gs call with them");
  if (!h->gs_flow || sc->waves <= 0)
    return fail(TR_ERR_UNSUPPORTED, "the allocation-free form runs the dataflow solves only (at most 15 sweeps)");
  const long long ncnt = sc->brick ? sc->nbricks : h->g.C;
  if (ncnt > kScratchCounters)
    return fail(TR_ERR_ARG, "the allocation-free coarse solve holds at most " + std::to_string(kScratchCounters) +
                                " update counters (" + std::to_string(ncnt) + " needed)");
  return translate([&]() {
    unsigned *base = scratch_ptr();
    int *err = reinterpret_cast<int *>(base);
    unsigned *cnt = base + kScratchHeader;
    DevLevel &D = h->lv[0];
    tr::launch_fill_u32(base, 1, S(st));  // error word (the counters are cleared by the launch)
    convert_in<double, double>(h, 0, adj, f, D.f64, S(st));
    if (sc->brick)
      tr::launch_coarse_brick(D.f64, D.u64, adj ? D.Gt64 : D.G64, h->sig_t, h->sig_s, D.ord, h->g, sc->wave_off,
                              sc->slots, sc->waves, adj, cnt, sc->nbricks, err, S(st));
    else
      tr::launch_coarse_flow(D.f64, D.u64, adj ? D.Gt64 : D.G64, h->sig_t, h->sig_s, D.ord, h->pl, h->g,
                             sc->wave_off, sc->slots, sc->waves, adj, cnt, err, S(st));
    tr::launch_convert<double, double>(D.u64, phi, D.P, h->g.S, adj ? D.winv : nullptr, nullptr, S(st));
    int e = 0;
    HIPCHK(hipMemcpyAsync(&e, err, sizeof(int), hipMemcpyDeviceToHost, S(st)));
    HIPCHK(hipStreamSynchronize(S(st)));
    if (e) throw std::runtime_error("coarse Gauss-Seidel solve timed out waiting for an upwind update");
    return TR_OK;
  });
}

int tr_mg_vcycle(tr_handle *h, int prec_mode, int adjoint, const double *r, double *z, tr_stream st) {
  if (!h || !r || !z) return fail(TR_ERR_ARG, "null argument");
  TR_CHECK_ALIGNED(r, z);
  if (!valid_mode(prec_mode)) return fail(TR_ERR_ARG, "bad preconditioner mode");
  return translate([&]() {
    precondition(h, prec_mode, adjoint != 0, r, z, S(st));
    check_barrier(h, S(st));
    return TR_OK;
  });
}

static int solve_common(tr_handle *h, bool adj, const double *b, double *x, const tr_solve_opts *o,
                        tr_solve_stats *stats, tr_stream st, bool bicg = false) {
  if (!h || !b || !x || !o || !stats) return fail(TR_ERR_ARG, "null argument");
  TR_CHECK_ALIGNED(b, x);
  if (o->restart < 1 || o->restart > 200 || o->max_restarts < 0 || !(o->tol > 0) || !valid_zstore(o->z_store))
    return fail(TR_ERR_ARG, "bad solver options");
  if (!valid_mode(o->prec_mode)) return fail(TR_ERR_ARG, "bad preconditioner mode");
  std::unique_ptr<EventTimer> timer;
  int rc = translate([&]() {
    if (o->timing) {
      timer.reset(new EventTimer());
      timer->on = true;
      timer->st = S(st);
      h->timer = timer.get();
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    h->n_precond = 0;
    h->sweep_dofs = 0;
    HIPCHK(hipEventRecord(e0, S(st)));
    int r = bicg ? bicgstab(h, adj, b, x, o, stats, S(st)) : gmres(h, adj, b, x, o, stats, S(st));
    HIPCHK(hipEventRecord(e1, S(st)));
    check_barrier(h, S(st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    fill_stats(h, stats, ms);
    h->timer = nullptr;
    return r;
  });
  h->timer = nullptr;
  if (rc == TR_ERR_NOCONV)
    g_err = bicg ? "BiCGStab reached its iteration limit before the tolerance"
                 : "GMRES reached max_restarts before the tolerance";
  return rc;
}

int tr_gmres_solve(tr_handle *h, const double *b, double *x, const tr_solve_opts *o, tr_solve_stats *stats,
                   tr_stream st) {
  return solve_common(h, false, b, x, o, stats, st);
}

int tr_bicgstab_solve(tr_handle *h, const double *b, double *x, const tr_solve_opts *o, tr_solve_stats *stats,
                      tr_stream st) {
  return solve_common(h, false, b, x, o, stats, st, true);
}

int tr_adjoint_grad(tr_handle *h, const double *w, const double *phi, double *lambda, double *grad_t, double *grad_s,
                    const tr_solve_opts *o, tr_solve_stats *stats, tr_stream st) {
  if (!h || !w || !phi || !grad_t || !grad_s || !o || !stats) return fail(TR_ERR_ARG, "null argument");
  TR_CHECK_ALIGNED(w, phi, lambda, grad_t, grad_s);
  double *lam = lambda;
  int rc = TR_OK;
  rc = translate([&]() {
    if (!lam) lam = h->kx ? h->kx : (h->kx = h->alloc<double>(h->vec_len(h->top())));
    return TR_OK;
  });
  if (rc) return rc;
  rc = solve_common(h, true, w, lam, o, stats, st);
  if (rc != TR_OK && rc != TR_ERR_NOCONV) return rc;
  int rc2 = translate([&]() {
    DevLevel &D = h->lv[h->top()];
    tr::launch_grad_t(lam, phi, D.w, D.P, h->g, grad_t, S(st));
    outer_scatter(h, phi, h->tmp, S(st));
    tr::launch_grad_s(lam, h->tmp, D.A, h->g, grad_s, S(st));
    HIPCHK(hipStreamSynchronize(S(st)));
    return TR_OK;
  });
  return rc2 ? rc2 : rc;
}

int tr_time_sweep_kernel(tr_handle *h, int level, int prec, int reps, double *ms, tr_stream st) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!ms || reps < 1) return fail(TR_ERR_ARG, "bad argument");
  return translate([&]() {
    DevLevel &D = h->lv[level];
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    if (prec == TR_F32) {
      if (level == 0) throw ArgError{"FP32 sweeps run on levels >= 1"};
      ensure_mixed(h);
      tr::launch_fill<float>(D.f32, h->vec_len(level), 1.0f, S(st));
      do_sweep<float>(h, level, D.f32, nullptr, D.u32, false, S(st));
      HIPCHK(hipEventRecord(e0, S(st)));
      for (int i = 0; i < reps; ++i) do_sweep<float>(h, level, D.f32, nullptr, D.u32, false, S(st));
    } else {
      do_sweep<double>(h, level, D.f64, nullptr, D.u64, false, S(st));
      HIPCHK(hipEventRecord(e0, S(st)));
      for (int i = 0; i < reps; ++i) do_sweep<double>(h, level, D.f64, nullptr, D.u64, false, S(st));
    }
    HIPCHK(hipEventRecord(e1, S(st)));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return TR_OK;
  });
}

int tr_time_scatter_kernel(tr_handle *h, int level, int outer, int prec, int reps, double *ms, tr_stream st) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!ms || reps < 1) return fail(TR_ERR_ARG, "bad argument");
  if (outer && level != h->top()) return fail(TR_ERR_ARG, "the problem operator lives on the finest level");
  return translate([&]() {
    DevLevel &D = h->lv[level];
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    if (prec == TR_F32 || prec == TR_F32_SPLIT) {
      if (level == 0) throw ArgError{"FP32 runs on levels >= 1"};
      ensure_mixed(h);
      // the level's scatter as the V-cycle runs it (TR_F32_SPLIT: with
      // split-BF16 products)
      auto run = [&]() {
        const bool keep = h->split32;
        h->split32 = prec == TR_F32_SPLIT;
        level_scatter<float>(h, level, false, D.u32, D.sa32, S(st));
        h->split32 = keep;
      };
      run();
      HIPCHK(hipEventRecord(e0, S(st)));
      for (int i = 0; i < reps; ++i) run();
    } else {
      auto run = [&]() {
        if (outer)
          outer_scatter(h, D.u64, D.sa64, S(st));
        else
          level_scatter<double>(h, level, false, D.u64, D.sa64, S(st));
      };
      run();
      HIPCHK(hipEventRecord(e0, S(st)));
      for (int i = 0; i < reps; ++i) run();
    }
    HIPCHK(hipEventRecord(e1, S(st)));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return TR_OK;
  });
}

}  // extern "C"
