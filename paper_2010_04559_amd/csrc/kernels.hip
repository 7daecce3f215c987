// Transport kernels for CDNA4 (gfx950): the ordinate-space DG transport
// sweep, the coarsest-level block Gauss-Seidel sweep, the problem-operator
// apply, basis conversions, inter-level transfers, sources and BLAS-1.
//
// Ordinate form.  With the collocated 3-point rule (points and weights w_k
// of each patch) the Lin coefficients phi_d of a patch and the values at its
// ordinates u_k are related by u = Psi phi, Psi = (3 I + J)/6 (symmetric).
// A weak-form right-hand side f of a patch becomes f^ = W^{-1} Psi^{-1} f,
// after which every (cell, ordinate) block of eq. complete is the upwind DG
// system of one discrete direction (local_solve.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>

#include "internal.h"
#include "local_solve.h"

namespace tr {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxMulti = 16;

__device__ __forceinline__ int insert_bit(int t, int d, int bit) {
  return (t & ((1 << d) - 1)) | (bit << d) | ((t >> d) << (d + 1));
}

template <typename T, int NS>
__device__ __forceinline__ void load_node_vec(const T *p, T *v) {
#pragma unroll
  for (int b = 0; b < NS; ++b) v[b] = p[b];
}

template <typename T, int NS>
__device__ __forceinline__ void store_node_vec(T *p, const T *v) {
#pragma unroll
  for (int b = 0; b < NS; ++b) p[b] = v[b];
}

__device__ __forceinline__ void unpack_cell(int packed, int flip, const Grid &g, int ci[3], int ix[3]) {
  ci[0] = packed & 1023;
  ci[1] = (packed >> 10) & 1023;
  ci[2] = (packed >> 20) & 1023;
#pragma unroll
  for (int d = 0; d < 3; ++d) ix[d] = ((flip >> d) & 1) ? g.n[d] - 1 - ci[d] : ci[d];
}

__device__ __forceinline__ long long cell_index(const int ix[3], const Grid &g) {
  return ix[0] + (long long)g.n[0] * (ix[1] + (long long)g.n[1] * ix[2]);
}

// Right-hand side of one ordinate's cell system, in the form solved by
// spectral_solve, from the cell's preloaded f and (optional) s values:
//   forward  v = f~ + sigma_s s + upwind inflow (scaled by N^{-1}), with the
//            prepared right-hand side f~ = N^{-1} f,
//   adjoint  v = f + sigma_s N s + downwind coupling.
template <typename T, int DIM, bool ADJ, int FLIP>
__device__ __forceinline__ void cell_rhs(T *v, const T *fv, const T *sv, bool has_s, const T *uk, const int ci[3],
                                         const int ix[3], const T *c, const T *a, double sigs, const Grid &g) {
  constexpr int flip = FLIP;
  constexpr int NS = 1 << DIM;
  // issue the neighbour-trace loads first (they are the only loads on the
  // sweep's dependence chain); a missing neighbour reads the cell itself
  // and is masked out below
  T tr[DIM][NS / 2];
  bool has[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int fl = (flip >> d) & 1;
    const int dir = fl ? -1 : 1;
    has[d] = ADJ ? (ci[d] < g.n[d] - 1) : (ci[d] > 0);
    int nx[3] = {ix[0], ix[1], ix[2]};
    if (has[d]) nx[d] += ADJ ? dir : -dir;
    const T *un = uk + cell_index(nx, g) * NS;
    // forward: the neighbour's outflow face; adjoint: its inflow face
    const int nbit = ADJ ? (fl ? 1 : 0) : (fl ? 0 : 1);
#pragma unroll
    for (int t = 0; t < NS / 2; ++t) tr[d][t] = un[insert_bit(t, d, nbit)];
  }
#pragma unroll
  for (int b = 0; b < NS; ++b) v[b] = fv[b];
  if (!ADJ) {
    if (has_s) {
#pragma unroll
      for (int b = 0; b < NS; ++b) v[b] += T(sigs) * sv[b];
    }
  } else if (has_s) {
    T t[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) t[b] = sv[b];
    mass_shape<T, DIM, false>(t);
    const T f = T(sigs * g.vol);
#pragma unroll
    for (int b = 0; b < NS; ++b) v[b] += f * t[b];
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    if (!has[d]) continue;
    const int fl = (flip >> d) & 1;
    if (!ADJ) {
      const int own0 = fl ? 1 : 0;   // own inflow face
#pragma unroll
      for (int t = 0; t < NS / 2; ++t) {
        v[insert_bit(t, d, own0)] += T(4) * c[d] * tr[d][t];
        v[insert_bit(t, d, 1 - own0)] -= T(2) * c[d] * tr[d][t];
      }
    } else {
      const int own1 = fl ? 0 : 1;   // own outflow face
      mass_shape<T, DIM - 1, false>(tr[d]);
      T hs = T(1);
#pragma unroll
      for (int e = 0; e < DIM; ++e)
        if (e != d) hs *= T(g.h[e]);
#pragma unroll
      for (int t = 0; t < NS / 2; ++t) v[insert_bit(t, d, own1)] += a[d] * hs * tr[d][t];
    }
  }
}

// ------------------------------------------------------------------ sweep
// One workgroup per ordinate walks the diagonal planes of its direction
// (downwind first for the adjoint); the cells of a plane are independent
// and each thread owns up to R of them.  The right-hand side and scatter
// source of the next plane do not depend on the sweep, so they are loaded
// into registers while the current plane is solved; only the upwind traces
// (written one plane earlier by this workgroup, L2-resident) sit on the
// dependence chain.
constexpr int kSweepThreads = 512;

// Body of the sweep for one ordinate whose octant sign bits FLIP are known
// at compile time, so every face-node index is a constant.
template <typename T, int DIM, bool ADJ, int R, bool PF, int FLIP>
__device__ __forceinline__ void sweep_body(const SweepArgs<T> &a, int k) {
  constexpr int NS = 1 << DIM;
  constexpr int RB = PF ? R : 1;  // register-buffered cells per thread
  constexpr int flip = FLIP;
  const OrdInfo o = a.ord[k];
  const T c[3] = {T(o.c[0]), T(o.c[1]), T(o.c[2])};
  const T av[3] = {T(o.a[0]), T(o.a[1]), T(o.a[2])};
  const long long S = a.g.S;
  const T *fk = a.f + (long long)k * S;
  const bool has_s = a.s != nullptr;
  const T *sk = has_s ? a.s + (long long)k * S : fk;
  T *uk = a.u + (long long)k * S;
  const int np = a.pl.nplanes;

  T fc[RB][NS], sc[RB][NS];
  auto load = [&](int pp, T (&fb)[RB][NS], T (&sb)[RB][NS]) {
    const int p = ADJ ? np - 1 - pp : pp;
    const int beg = a.pl.off[p], end = a.pl.off[p + 1];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int idx = beg + threadIdx.x + r * kSweepThreads;
      if (idx < end) {
        int ci[3], ix[3];
        unpack_cell(a.pl.cells[idx], flip, a.g, ci, ix);
        const long long j = cell_index(ix, a.g);
        load_node_vec<T, NS>(fk + j * NS, fb[r]);
        if (has_s) load_node_vec<T, NS>(sk + j * NS, sb[r]);
      }
    }
  };
  if (PF) load(0, fc, sc);
  for (int pp = 0; pp < np; ++pp) {
    T fn[RB][NS], sn[RB][NS];
    if (PF && pp + 1 < np) load(pp + 1, fn, sn);
    const int p = ADJ ? np - 1 - pp : pp;
    const int beg = a.pl.off[p], end = a.pl.off[p + 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int idx = beg + threadIdx.x + r * kSweepThreads;
      if (idx < end) {
        int ci[3], ix[3];
        unpack_cell(a.pl.cells[idx], flip, a.g, ci, ix);
        const long long j = cell_index(ix, a.g);
        T v[NS];
        if (PF) {
          cell_rhs<T, DIM, ADJ, FLIP>(v, fc[PF ? r : 0], sc[PF ? r : 0], has_s, uk, ci, ix, c, av, a.sig_s[j], a.g);
        } else {
          T fv[NS], sv[NS];
          load_node_vec<T, NS>(fk + j * NS, fv);
          if (has_s) load_node_vec<T, NS>(sk + j * NS, sv);
          cell_rhs<T, DIM, ADJ, FLIP>(v, fv, sv, has_s, uk, ci, ix, c, av, a.sig_s[j], a.g);
        }
        spectral_solve<T, DIM, ADJ>(v, c, T(a.sig_t[j]), flip);
        if (ADJ) {
          mass_shape<T, DIM, true>(v);
          const T iv = T(1.0 / a.g.vol);
#pragma unroll
          for (int b = 0; b < NS; ++b) v[b] *= iv;
        }
        store_node_vec<T, NS>(uk + j * NS, v);
      }
    }
    __syncthreads();
    if (PF) {
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int b = 0; b < NS; ++b) {
          fc[r][b] = fn[r][b];
          sc[r][b] = sn[r][b];
        }
    }
  }
}

template <typename T, int DIM, bool ADJ, int R, bool PF>
__global__ __launch_bounds__(kSweepThreads) void k_sweep(SweepArgs<T> a) {
  const int k = blockIdx.x;
  switch (a.ord[k].flip) {
    case 0: sweep_body<T, DIM, ADJ, R, PF, 0>(a, k); break;
    case 1: sweep_body<T, DIM, ADJ, R, PF, 1>(a, k); break;
    case 2: sweep_body<T, DIM, ADJ, R, PF, 2>(a, k); break;
    case 3: sweep_body<T, DIM, ADJ, R, PF, 3>(a, k); break;
    case 4: if (DIM == 3) sweep_body<T, DIM, ADJ, R, PF, 4>(a, k); break;
    case 5: if (DIM == 3) sweep_body<T, DIM, ADJ, R, PF, 5>(a, k); break;
    case 6: if (DIM == 3) sweep_body<T, DIM, ADJ, R, PF, 6>(a, k); break;
    default: if (DIM == 3) sweep_body<T, DIM, ADJ, R, PF, 7>(a, k); break;
  }
}

// ------------------------------------------------------------ LDS sweep
// The same sweep with the previous plane's solution kept in LDS (node-major,
// [node][position in plane]), so that the dependence chain from one plane
// to the next never leaves the CU.  A 1024-thread workgroup per ordinate is
// split into compute waves (one cell per thread and plane) and store waves.
//  * Global memory is accessed in whole cells: a 16-byte load or store of
//    a wave covers 64 / Q cells completely (Q = 16-byte chunks per cell),
//    instead of one chunk of 64 different cells.  Loaded chunks are moved
//    to the thread that owns the cell through a per-wave LDS staging area.
//  * Compute waves issue only loads: the next plane's right-hand side (and
//    scatter source), cross sections and, one plane further ahead, its
//    cell-list entries are loaded while the current plane is solved and
//    awaited only after the plane's barriers.
//  * Store waves copy each finished plane from LDS to global memory, so no
//    compute wave ever waits for a store (gfx9 counts loads and stores on
//    one counter, so a wait for a load would include every earlier store).
// Planes alternate between two LDS buffers where they fit, and each plane
// then takes one workgroup barrier (waiting for LDS traffic only) before
// the next plane and the store waves read it: a plane's values overwrite
// those of two planes back, whose readers all passed the barrier between.
// With one buffer a second barrier precedes the overwrite.

__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ long long flipped_cell(int packed, int flip, const Grid &g) {
  int ci[3], ix[3];
  unpack_cell(packed, flip, g, ci, ix);
  return cell_index(ix, g);
}

// Marks a register as used at this point (an empty asm statement): the
// compiler must wait here for a load that produces it, and cannot move the
// wait before an earlier barrier.
__device__ __forceinline__ void pin_reg(float4 &x) {
  asm volatile("" : "+v"(x.x), "+v"(x.y), "+v"(x.z), "+v"(x.w));
}
__device__ __forceinline__ void pin_reg(int4 &x) {
  asm volatile("" : "+v"(x.x), "+v"(x.y), "+v"(x.z), "+v"(x.w));
}
__device__ __forceinline__ void pin_reg(double &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin_reg(int &x) { asm volatile("" : "+v"(x)); }

// Staged next-plane data of a compute lane: Q 16-byte chunks of f (and s)
// as loaded (chunk l / CPI of the wave's cell CPI i + l % CPI for chunk
// slot i), and the lane's own cross sections and cell-list entry.
template <int Q, bool HAS_S>
struct StageRegs {
  float4 f[Q], s[HAS_S ? Q : 1];
  double st, ss;
  int4 lk;
};

// One cell per compute lane (planes up to 960 cells), 1024 threads.
template <typename T, int DIM, bool ADJ, bool HAS_S, bool DBUF, bool PIN, int FLIP>
__device__ __forceinline__ void sweep_lds_body1(const SweepArgs<T> &a, int k, T *lds, int *jbuf, const int *off,
                                               float4 *stage, int tc) {
  constexpr int NS = 1 << DIM;
  constexpr int Q = NS * (int)sizeof(T) / 16;  // 16-byte chunks per cell
  constexpr int CPI = 64 / Q;                   // cells per 16-byte wave access
  constexpr int EPC = 16 / (int)sizeof(T);      // elements per chunk
  using Regs = StageRegs<Q, HAS_S>;
  const OrdInfo o = a.ord[k];
  const T c[3] = {T(o.c[0]), T(o.c[1]), T(o.c[2])};
  const T av[3] = {T(o.a[0]), T(o.a[1]), T(o.a[2])};
  const ModeConst<T, DIM> mc = mode_const<T, DIM>(c);
  const long long S = a.g.S;
  const T *fk = a.f + (long long)k * S;
  const T *sk = HAS_S ? a.s + (long long)k * S : nullptr;
  T *uk = a.u + (long long)k * S;
  const long long C = a.g.C;
  const double *sgt = a.sig_pl + (long long)FLIP * C;
  const double *sgs = a.sig_pl + (8LL + FLIP) * C;
  const int np = a.pl.nplanes;
  const int maxp = a.pl.max_plane;
  const int4 *link = a.pl.link[ADJ ? 1 : 0];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const bool compute = tid < tc;
  // this wave's staging area: Q KB for f, then Q KB for s
  float4 *stg = stage + (size_t)(tid >> 6) * (HAS_S ? 2 : 1) * Q * 64;
  auto plane_of = [&](int pp) { return ADJ ? np - 1 - pp : pp; };
  // Every global load below is unconditional, from an address clamped to
  // valid memory, and its validity is applied only after the wait: a load
  // under a branch, or a select on its result, would make the compiler
  // wait for it (and for everything issued before it) at once.
  auto link_valid = [&](int pp) {
    const int p = plane_of(pp);
    return off[p] + tid < off[p + 1];
  };
  auto load_link = [&](int pp) {
    const int p = plane_of(pp);
    return link[min(off[p] + tid, (int)C - 1)];
  };
  // loads of plane pp for this wave's 64 cells; q.lk holds the lane's own
  // entry (its cell index is shuffled to the lanes that load its chunks)
  auto load_plane = [&](int pp, Regs &q) {
    const int p = plane_of(pp);
    const int idx = min(off[p] + tid, (int)C - 1);
    const int j = q.lk.x >= 0 ? (int)flipped_cell(q.lk.x, FLIP, a.g) : 0;
    const int ch = lane / CPI;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int jj = __shfl(j, CPI * i + lane % CPI, 64);
      // plane layout: the wave's cells are consecutive list positions
      const long long fi = PIN ? (long long)min(off[p] + (tid & ~63) + CPI * i + lane % CPI, (int)C - 1) : jj;
      q.f[i] = *reinterpret_cast<const float4 *>(fk + fi * NS + ch * EPC);
      if (HAS_S) q.s[HAS_S ? i : 0] = *reinterpret_cast<const float4 *>(sk + (long long)jj * NS + ch * EPC);
    }
    q.st = sgt[idx];
    if (HAS_S) q.ss = sgs[idx];
  };
  // staged chunks -> LDS staging (same wave writes and reads it)
  auto stage_plane = [&](Regs &q) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      stg[i * 64 + lane] = q.f[i];
      if (HAS_S) stg[(Q + i) * 64 + lane] = q.s[HAS_S ? i : 0];
    }
  };
  auto read_cell = [&](T *fv, T *sv) {
    const int i = lane / CPI, cc = lane % CPI;
#pragma unroll
    for (int ch = 0; ch < Q; ++ch) {
      const float4 x = stg[i * 64 + ch * CPI + cc];
      const T *xe = reinterpret_cast<const T *>(&x);
#pragma unroll
      for (int e = 0; e < EPC; ++e) fv[ch * EPC + e] = xe[e];
      if (HAS_S) {
        const float4 y = stg[(Q + i) * 64 + ch * CPI + cc];
        const T *ye = reinterpret_cast<const T *>(&y);
#pragma unroll
        for (int e = 0; e < EPC; ++e) sv[ch * EPC + e] = ye[e];
      }
    }
  };

  Regs cur, nxt;
  cur.lk = make_int4(-1, -1, -1, -1);
  nxt.lk = make_int4(-1, -1, -1, -1);
  if (compute) {
    cur.lk = load_link(0);
    pin_reg(cur.lk);
    if (!link_valid(0)) cur.lk.x = -1;
    load_plane(0, cur);
    nxt.lk = load_link(min(1, np - 1));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      pin_reg(cur.f[i]);
      if (HAS_S) pin_reg(cur.s[HAS_S ? i : 0]);
    }
    pin_reg(cur.st);
    if (HAS_S) pin_reg(cur.ss);
    pin_reg(nxt.lk);
    if (np < 2 || !link_valid(1)) nxt.lk.x = -1;
    stage_plane(cur);
  }

  // Compute and store waves run separate loops with the same two barriers
  // per plane (a workgroup barrier counts waves, not program locations).
  // Inside the compute loop nothing branches around the loads or between
  // them and their waits, so no load is awaited early.
  if (compute) {
    for (int pp = 0; pp < np; ++pp) {
      const bool mine = cur.lk.x >= 0;
      // part of the right-hand side independent of the sweep: forward, the
      // prepared right-hand side itself (f~ = N^{-1} f, or f~ + sigma_s G u
      // formed by the scatter GEMM); adjoint  v = f + sigma_s N s
      T v[NS], sv[NS];
      read_cell(v, sv);
      if (!ADJ && HAS_S) {
#pragma unroll
        for (int b = 0; b < NS; ++b) v[b] += T(cur.ss) * sv[b];
      } else if (ADJ && HAS_S) {
        mass_shape<T, DIM, false>(sv);
        const T fs = T(cur.ss) * T(a.g.vol);
#pragma unroll
        for (int b = 0; b < NS; ++b) v[b] += fs * sv[b];
      }
      // (past the last plane the last one is loaded again, unused)
      load_plane(min(pp + 1, np - 1), nxt);
      int4 lk2 = load_link(min(pp + 2, np - 1));
      // neighbour traces from LDS: forward, the upwind neighbour's outflow
      // face; adjoint, the downwind neighbour's inflow face (cells without
      // a neighbour, or lanes without a cell, read position 0 and drop it)
      const int nbp[3] = {cur.lk.y, cur.lk.z, cur.lk.w};
      const T *rd = lds + (DBUF ? ((pp + 1) & 1) : 0) * NS * maxp;  // previous plane
      T tr[DIM][NS / 2];
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int fl = (FLIP >> d) & 1;
        const int nbit = ADJ ? (fl ? 1 : 0) : (fl ? 0 : 1);
        const int q = nbp[d] >= 0 ? nbp[d] : 0;
#pragma unroll
        for (int t = 0; t < NS / 2; ++t) {
          const T x = rd[insert_bit(t, d, nbit) * maxp + q];  // may be uninitialised: select, not scale
          tr[d][t] = nbp[d] >= 0 ? x : T(0);
        }
      }
      if (!ADJ) {
        // inflow: 4 c on the own inflow face, -2 c on the opposite face
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const int own0 = (FLIP >> d) & 1;
          const T c4 = T(4) * c[d], c2 = T(2) * c[d];
#pragma unroll
          for (int t = 0; t < NS / 2; ++t) {
            v[insert_bit(t, d, own0)] += c4 * tr[d][t];
            v[insert_bit(t, d, 1 - own0)] -= c2 * tr[d][t];
          }
        }
      } else {
        // outflow coupling a_xi (face mass) on the own outflow face
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const int own1 = ((FLIP >> d) & 1) ? 0 : 1;
          mass_shape<T, DIM - 1, false>(tr[d]);
          T hs = av[d];
#pragma unroll
          for (int e = 0; e < DIM; ++e)
            if (e != d) hs *= T(a.g.h[e]);
#pragma unroll
          for (int t = 0; t < NS / 2; ++t) v[insert_bit(t, d, own1)] += hs * tr[d][t];
        }
      }
      oriented_solve<T, DIM, ADJ, FLIP>(v, mc, T(cur.st));
      if (ADJ) {
        mass_shape<T, DIM, true>(v);
        const T iv = T(1.0 / a.g.vol);
#pragma unroll
        for (int b = 0; b < NS; ++b) v[b] *= iv;
      }
      // single buffer: every read of the previous plane must be done first;
      // double buffer: the plane goes to the other buffer
      if (!DBUF) lds_barrier();
      if (mine) {
        T *wr = lds + (DBUF ? (pp & 1) : 0) * NS * maxp;
#pragma unroll
        for (int b = 0; b < NS; ++b) wr[b * maxp + tid] = v[b];
        jbuf[(DBUF ? (pp & 1) : 0) * maxp + tid] = (int)flipped_cell(cur.lk.x, FLIP, a.g);
      }
      lds_barrier();  // the plane is complete in LDS
      // the next plane's loads are awaited only now, after both barriers
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        pin_reg(nxt.f[i]);
        if (HAS_S) pin_reg(nxt.s[HAS_S ? i : 0]);
      }
      pin_reg(nxt.st);
      if (HAS_S) pin_reg(nxt.ss);
      pin_reg(lk2);
      stage_plane(nxt);
      if (pp + 2 >= np || !link_valid(pp + 2)) lk2.x = -1;
      cur = nxt;
      nxt.lk = lk2;
    }
  } else {
    // store waves: chunk lane / CPI of cell CPI i + lane % CPI of each
    // group of 64 cells, whole cells per access
    const int ch = lane / CPI;
    for (int pp = 0; pp < np; ++pp) {
      if (!DBUF) lds_barrier();
      lds_barrier();
      const int p = plane_of(pp);
      const int n = off[p + 1] - off[p];
      const T *pb = lds + (DBUF ? (pp & 1) : 0) * NS * maxp;
      const int *jb = jbuf + (DBUF ? (pp & 1) : 0) * maxp;
      for (int base = (tid - tc) / 64 * CPI; base < n; base += (1024 - tc) / 64 * CPI) {
        const int q = base + lane % CPI;
        if (q < n) {
          T w[EPC];
#pragma unroll
          for (int e = 0; e < EPC; ++e) w[e] = pb[(ch * EPC + e) * maxp + q];
          *reinterpret_cast<float4 *>(uk + (long long)jb[q] * NS + ch * EPC) = *reinterpret_cast<float4 *>(w);
        }
      }
    }
  }
}

// Several cells per compute lane (larger planes; FP32, 3-D).
template <typename T, int DIM, bool ADJ, bool HAS_S, bool DBUF, bool PIN, int FLIP, int CPT, int NT>
__device__ __forceinline__ void sweep_lds_body(const SweepArgs<T> &a, int k, T *lds, int *jbuf, const int *off,
                                               float4 *stage, int tc) {
  constexpr int NS = 1 << DIM;
  constexpr int Q = NS * (int)sizeof(T) / 16;  // 16-byte chunks per cell
  constexpr int CPI = 64 / Q;                   // cells per 16-byte wave access
  constexpr int EPC = 16 / (int)sizeof(T);      // elements per chunk
  using Regs = StageRegs<Q, HAS_S>;
  const OrdInfo o = a.ord[k];
  const T c[3] = {T(o.c[0]), T(o.c[1]), T(o.c[2])};
  const T av[3] = {T(o.a[0]), T(o.a[1]), T(o.a[2])};
  const ModeConst<T, DIM> mc = mode_const<T, DIM>(c);
  const long long S = a.g.S;
  const T *fk = a.f + (long long)k * S;
  const T *sk = HAS_S ? a.s + (long long)k * S : nullptr;
  T *uk = a.u + (long long)k * S;
  const long long C = a.g.C;
  const double *sgt = a.sig_pl + (long long)FLIP * C;
  const double *sgs = a.sig_pl + (8LL + FLIP) * C;
  const int np = a.pl.nplanes;
  const int maxp = a.pl.max_plane;
  const int4 *link = a.pl.link[ADJ ? 1 : 0];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const bool compute = tid < tc;
  // this wave's staging area: Q KB for f, then Q KB for s (the CPT cell
  // groups of a lane pass through it one after the other)
  float4 *stg = stage + (size_t)(tid >> 6) * (HAS_S ? 2 : 1) * Q * 64;
  auto plane_of = [&](int pp) { return ADJ ? np - 1 - pp : pp; };
  // Every global load below is unconditional, from an address clamped to
  // valid memory, and its validity is applied only after the wait: a load
  // under a branch, or a select on its result, would make the compiler
  // wait for it (and for everything issued before it) at once.  Cell group
  // r of a compute lane is plane position tid + r tc.
  auto link_valid = [&](int pp, int r) {
    const int p = plane_of(pp);
    return off[p] + tid + r * tc < off[p + 1];
  };
  auto load_link = [&](int pp, int r) {
    const int p = plane_of(pp);
    return link[min(off[p] + tid + r * tc, (int)C - 1)];
  };
  // loads of plane pp for this wave's 64 cells of group r; q.lk holds the
  // lane's own entry (its cell index is shuffled to the lanes that load
  // its chunks)
  auto load_plane = [&](int pp, int r, Regs &q) {
    const int p = plane_of(pp);
    const int idx = min(off[p] + tid + r * tc, (int)C - 1);
    const int j = q.lk.x >= 0 ? (int)flipped_cell(q.lk.x, FLIP, a.g) : 0;
    const int ch = lane / CPI;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int jj = __shfl(j, CPI * i + lane % CPI, 64);
      // plane layout: the wave's cells are consecutive list positions
      const long long fi =
          PIN ? (long long)min(off[p] + (tid & ~63) + r * tc + CPI * i + lane % CPI, (int)C - 1) : jj;
      q.f[i] = *reinterpret_cast<const float4 *>(fk + fi * NS + ch * EPC);
      if (HAS_S) q.s[HAS_S ? i : 0] = *reinterpret_cast<const float4 *>(sk + (long long)jj * NS + ch * EPC);
    }
    q.st = sgt[idx];
    if (HAS_S) q.ss = sgs[idx];
  };
  // staged chunks -> LDS staging (same wave writes and reads it)
  auto stage_plane = [&](Regs &q) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      stg[i * 64 + lane] = q.f[i];
      if (HAS_S) stg[(Q + i) * 64 + lane] = q.s[HAS_S ? i : 0];
    }
  };
  auto read_cell = [&](T *fv, T *sv) {
    const int i = lane / CPI, cc = lane % CPI;
#pragma unroll
    for (int ch = 0; ch < Q; ++ch) {
      const float4 x = stg[i * 64 + ch * CPI + cc];
      const T *xe = reinterpret_cast<const T *>(&x);
#pragma unroll
      for (int e = 0; e < EPC; ++e) fv[ch * EPC + e] = xe[e];
      if (HAS_S) {
        const float4 y = stg[(Q + i) * 64 + ch * CPI + cc];
        const T *ye = reinterpret_cast<const T *>(&y);
#pragma unroll
        for (int e = 0; e < EPC; ++e) sv[ch * EPC + e] = ye[e];
      }
    }
  };
  auto pin_regs = [&](Regs &q) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      pin_reg(q.f[i]);
      if (HAS_S) pin_reg(q.s[HAS_S ? i : 0]);
    }
    pin_reg(q.st);
    if (HAS_S) pin_reg(q.ss);
  };

  Regs cur[CPT], nxt[CPT];
#pragma unroll
  for (int r = 0; r < CPT; ++r) {
    cur[r].lk = make_int4(-1, -1, -1, -1);
    nxt[r].lk = make_int4(-1, -1, -1, -1);
  }
  if (compute) {
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      cur[r].lk = load_link(0, r);
      pin_reg(cur[r].lk);
      if (!link_valid(0, r)) cur[r].lk.x = -1;
      load_plane(0, r, cur[r]);
      nxt[r].lk = load_link(min(1, np - 1), r);
    }
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      pin_regs(cur[r]);
      pin_reg(nxt[r].lk);
      if (np < 2 || !link_valid(1, r)) nxt[r].lk.x = -1;
    }
    stage_plane(cur[0]);
  }

  // Compute and store waves run separate loops with the same barriers per
  // plane (a workgroup barrier counts waves, not program locations).
  // Inside the compute loop nothing branches around the loads or between
  // them and their waits, so no load is awaited early.
  if (compute) {
    for (int pp = 0; pp < np; ++pp) {
      int4 lk2[CPT];
      const T *rd = lds + (DBUF ? ((pp + 1) & 1) : 0) * NS * maxp;  // previous plane
      T *wr = lds + (DBUF ? (pp & 1) : 0) * NS * maxp;
      T res[DBUF ? 1 : CPT][NS];  // single buffer: results held until every read is done
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        // part of the right-hand side independent of the sweep: forward,
        // the prepared right-hand side itself (f~ = N^{-1} f, or f~ +
        // sigma_s G u formed by the scatter GEMM); adjoint v = f + sigma_s N s
        if (r > 0) stage_plane(cur[r]);
        T v[NS], sv[NS];
        read_cell(v, sv);
        if (!ADJ && HAS_S) {
#pragma unroll
          for (int b = 0; b < NS; ++b) v[b] += T(cur[r].ss) * sv[b];
        } else if (ADJ && HAS_S) {
          mass_shape<T, DIM, false>(sv);
          const T fs = T(cur[r].ss) * T(a.g.vol);
#pragma unroll
          for (int b = 0; b < NS; ++b) v[b] += fs * sv[b];
        }
        if (r == 0) {
          // the next plane's loads, in flight during this plane's work
          // (past the last plane the last one is loaded again, unused)
#pragma unroll
          for (int r2 = 0; r2 < CPT; ++r2) {
            load_plane(min(pp + 1, np - 1), r2, nxt[r2]);
            lk2[r2] = load_link(min(pp + 2, np - 1), r2);
          }
        }
        // neighbour traces from LDS: forward, the upwind neighbour's
        // outflow face; adjoint, the downwind neighbour's inflow face
        // (cells without a neighbour, or lanes without a cell, read
        // position 0 and drop it)
        const int nbp[3] = {cur[r].lk.y, cur[r].lk.z, cur[r].lk.w};
        T tr[DIM][NS / 2];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const int fl = (FLIP >> d) & 1;
          const int nbit = ADJ ? (fl ? 1 : 0) : (fl ? 0 : 1);
          const int q = nbp[d] >= 0 ? nbp[d] : 0;
#pragma unroll
          for (int t = 0; t < NS / 2; ++t) {
            const T x = rd[insert_bit(t, d, nbit) * maxp + q];  // may be uninitialised: select, not scale
            tr[d][t] = nbp[d] >= 0 ? x : T(0);
          }
        }
        if (!ADJ) {
          // inflow: 4 c on the own inflow face, -2 c on the opposite face
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            const int own0 = (FLIP >> d) & 1;
            const T c4 = T(4) * c[d], c2 = T(2) * c[d];
#pragma unroll
            for (int t = 0; t < NS / 2; ++t) {
              v[insert_bit(t, d, own0)] += c4 * tr[d][t];
              v[insert_bit(t, d, 1 - own0)] -= c2 * tr[d][t];
            }
          }
        } else {
          // outflow coupling a_xi (face mass) on the own outflow face
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            const int own1 = ((FLIP >> d) & 1) ? 0 : 1;
            mass_shape<T, DIM - 1, false>(tr[d]);
            T hs = av[d];
#pragma unroll
            for (int e = 0; e < DIM; ++e)
              if (e != d) hs *= T(a.g.h[e]);
#pragma unroll
            for (int t = 0; t < NS / 2; ++t) v[insert_bit(t, d, own1)] += hs * tr[d][t];
          }
        }
        oriented_solve<T, DIM, ADJ, FLIP>(v, mc, T(cur[r].st));
        if (ADJ) {
          mass_shape<T, DIM, true>(v);
          const T iv = T(1.0 / a.g.vol);
#pragma unroll
          for (int b = 0; b < NS; ++b) v[b] *= iv;
        }
        if (DBUF) {
          // the plane goes to the other buffer: write at once
          if (cur[r].lk.x >= 0) {
#pragma unroll
            for (int b = 0; b < NS; ++b) wr[b * maxp + tid + r * tc] = v[b];
            jbuf[(pp & 1) * maxp + tid + r * tc] = (int)flipped_cell(cur[r].lk.x, FLIP, a.g);
          }
        } else {
#pragma unroll
          for (int b = 0; b < NS; ++b) res[DBUF ? 0 : r][b] = v[b];
        }
      }
      if (!DBUF) {
        // single buffer: every read of the previous plane must be done first
        lds_barrier();
#pragma unroll
        for (int r = 0; r < CPT; ++r)
          if (cur[r].lk.x >= 0) {
#pragma unroll
            for (int b = 0; b < NS; ++b) wr[b * maxp + tid + r * tc] = res[DBUF ? 0 : r][b];
            jbuf[tid + r * tc] = (int)flipped_cell(cur[r].lk.x, FLIP, a.g);
          }
      }
      lds_barrier();  // the plane is complete in LDS
      // the next plane's loads are awaited only now, after the barriers
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        pin_regs(nxt[r]);
        pin_reg(lk2[r]);
      }
      stage_plane(nxt[0]);
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        if (pp + 2 >= np || !link_valid(pp + 2, r)) lk2[r].x = -1;
        cur[r] = nxt[r];
        nxt[r].lk = lk2[r];
      }
    }
  } else {
    // store waves: chunk lane / CPI of cell CPI i + lane % CPI of each
    // group of 64 cells, whole cells per access
    const int ch = lane / CPI;
    for (int pp = 0; pp < np; ++pp) {
      if (!DBUF) lds_barrier();
      lds_barrier();
      const int p = plane_of(pp);
      const int n = off[p + 1] - off[p];
      const T *pb = lds + (DBUF ? (pp & 1) : 0) * NS * maxp;
      const int *jb = jbuf + (DBUF ? (pp & 1) : 0) * maxp;
      for (int base = (tid - tc) / 64 * CPI; base < n; base += (NT - tc) / 64 * CPI) {
        const int q = base + lane % CPI;
        if (q < n) {
          T w[EPC];
#pragma unroll
          for (int e = 0; e < EPC; ++e) w[e] = pb[(ch * EPC + e) * maxp + q];
          *reinterpret_cast<float4 *>(uk + (long long)jb[q] * NS + ch * EPC) = *reinterpret_cast<float4 *>(w);
        }
      }
    }
  }
}

template <typename T, int DIM, bool ADJ, bool HAS_S, bool DBUF, bool PIN, int CPT, int NT>
__global__ __launch_bounds__(NT) void k_sweep_lds(SweepArgs<T> a, int tc) {
  extern __shared__ __align__(16) unsigned char sweep_smem[];
  constexpr int NS = 1 << DIM;
  constexpr int Q = NS * (int)sizeof(T) / 16;
  float4 *stage = reinterpret_cast<float4 *>(sweep_smem);
  T *lds = reinterpret_cast<T *>(stage + (size_t)(tc / 64) * (HAS_S ? 2 : 1) * Q * 64);
  constexpr int NB = DBUF ? 2 : 1;  // plane buffers
  int *jbuf = reinterpret_cast<int *>(lds + (size_t)NB * NS * a.pl.max_plane);
  // plane offsets in LDS: read with LDS loads, they never make a compute
  // wave wait on the vector-memory counter
  int *off = jbuf + NB * a.pl.max_plane;
  for (int i = threadIdx.x; i <= a.pl.nplanes; i += blockDim.x) off[i] = a.pl.off[i];
  __syncthreads();
  const int k = blockIdx.x;
#define TR_SWEEP_LDS(F)                                                                     \
  if constexpr (CPT == 1)                                                                   \
    sweep_lds_body1<T, DIM, ADJ, HAS_S, DBUF, PIN, F>(a, k, lds, jbuf, off, stage, tc);     \
  else                                                                                      \
    sweep_lds_body<T, DIM, ADJ, HAS_S, DBUF, PIN, F, CPT, NT>(a, k, lds, jbuf, off, stage, tc)
  switch (a.ord[k].flip) {
    case 0: TR_SWEEP_LDS(0); break;
    case 1: TR_SWEEP_LDS(1); break;
    case 2: TR_SWEEP_LDS(2); break;
    case 3: TR_SWEEP_LDS(3); break;
    case 4: if (DIM == 3) TR_SWEEP_LDS(4); break;
    case 5: if (DIM == 3) TR_SWEEP_LDS(5); break;
    case 6: if (DIM == 3) TR_SWEEP_LDS(6); break;
    default: if (DIM == 3) TR_SWEEP_LDS(7); break;
  }
#undef TR_SWEEP_LDS
}

// ------------------------------------------------------------ pair sweep
// The forward 3-D sweep over bricks of two x-adjacent cells: cells 2b and
// 2b + 1 of the sweep frame, which reflection keeps an aligned pair of
// memory when the grid has an even number of cells along x.  Bricks are
// walked in the diagonal planes of the brick grid (b + iy + iz); a lane
// solves its brick's two cells in sweep order, the second taking its x
// inflow from the first in registers, and the previous plane's bricks are
// kept in LDS as in the cell kernel above.  A brick's values are 2 ns
// contiguous elements (64 bytes in FP32, 128 in FP64), so every global
// access moves whole 64-byte units: FP32 cells written one at a time are
// 32-byte partial writes, which the memory serves at a fraction of the
// rate of whole units (measured: those stores took 60% of the cell
// kernel's time at 48^3).
// Inputs in plane layout hold brick i's cells at positions 2i and 2i + 1
// (slot order: slot 0 is the upwind cell); in spatial order the pair is
// read as stored (physical x order) and mapped to slots.  Each lane loads
// its brick's chunks itself (no staging: the brick is one aligned unit).
// LDS: [buffer][slot][node][brick position] values, per buffer the first
// (lower-address) cell of each brick of the plane, then the plane offsets.

template <typename T, bool HAS_S>
struct PairRegs {
  static constexpr int PQ = 2 * 8 * (int)sizeof(T) / 16;  // 16-byte chunks per brick
  float4 f[PQ], s[HAS_S ? PQ : 1];
  double2 st, ss;  // cross sections of slots 0 and 1
  int4 lk;
};

template <typename T, bool HAS_S>
__device__ __forceinline__ void pin_regs_pair(PairRegs<T, HAS_S> &q) {
#pragma unroll
  for (int i = 0; i < PairRegs<T, HAS_S>::PQ; ++i) {
    pin_reg(q.f[i]);
    if (HAS_S) pin_reg(q.s[HAS_S ? i : 0]);
  }
  pin_reg(q.st.x);
  pin_reg(q.st.y);
  if (HAS_S) {
    pin_reg(q.ss.x);
    pin_reg(q.ss.y);
  }
}

// element m (0 .. 2 ns - 1, memory order of the brick) of a chunk array
template <typename T, int N>
__device__ __forceinline__ T pair_elem(const float4 (&arr)[N], int m) {
  constexpr int EPC = 16 / (int)sizeof(T);
  const float4 x = arr[m / EPC];
  return reinterpret_cast<const T *>(&x)[m % EPC];
}

template <typename T, bool HAS_S, bool DBUF, bool PIN, int FLIP, int CPT, int NT>
__device__ __forceinline__ void sweep_pair_body(const SweepArgs<T> &a, int k, T *lds, int *jbuf, const int *off,
                                                int tc) {
  constexpr int NS = 8;
  constexpr int EPC = 16 / (int)sizeof(T);
  using Regs = PairRegs<T, HAS_S>;
  constexpr int PQ = Regs::PQ;
  constexpr int FX = FLIP & 1;  // x reflected: slot 0 is the pair's upper cell in memory
  const OrdInfo o = a.ord[k];
  const T c[3] = {T(o.c[0]), T(o.c[1]), T(o.c[2])};
  const ModeConst<T, 3> mc = mode_const<T, 3>(c);
  const long long S = a.g.S;
  const T *fk = a.f + (long long)k * S;
  const T *sk = HAS_S ? a.s + (long long)k * S : nullptr;
  T *uk = a.u + (long long)k * S;
  const long long C = a.g.C;
  const int nbr = (int)(C / 2);  // bricks
  const double *sgt = a.sig_pb + (long long)FLIP * C;
  const double *sgs = a.sig_pb + (8LL + FLIP) * C;
  const int np = a.bpl.nplanes;
  const int maxp = a.bpl.max_plane;
  const int4 *link = a.bpl.link[0];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const bool compute = tid < tc;
  // lower-address cell of the brick packed bp in this orientation
  auto base_cell = [&](int bp) -> long long {
    const int bx = bp & 1023, iy = (bp >> 10) & 1023, iz = (bp >> 20) & 1023;
    const int ix = (FLIP & 1) ? a.g.n[0] - 2 - 2 * bx : 2 * bx;
    const int jy = (FLIP & 2) ? a.g.n[1] - 1 - iy : iy;
    const int jz = (FLIP & 4) ? a.g.n[2] - 1 - iz : iz;
    return ix + (long long)a.g.n[0] * (jy + (long long)a.g.n[1] * jz);
  };
  // As in the cell kernels: every global load is unconditional, from an
  // address clamped to valid memory, its validity applied after the wait.
  // Brick group r of a compute lane is plane position tid + r tc.
  auto link_valid = [&](int pp, int r) { return off[pp] + tid + r * tc < off[pp + 1]; };
  auto load_link = [&](int pp, int r) { return link[min(off[pp] + tid + r * tc, nbr - 1)]; };
  auto load_plane = [&](int pp, int r, Regs &q) {
    const int bi = min(off[pp] + tid + r * tc, nbr - 1);
    const long long jb = base_cell(q.lk.x >= 0 ? q.lk.x : 0);
    const float4 *src = reinterpret_cast<const float4 *>(fk + (PIN ? 2LL * bi : jb) * NS);
#pragma unroll
    for (int i = 0; i < PQ; ++i) q.f[i] = src[i];
    if (HAS_S) {
      const float4 *ss = reinterpret_cast<const float4 *>(sk + jb * NS);
#pragma unroll
      for (int i = 0; i < PQ; ++i) q.s[HAS_S ? i : 0] = ss[i];
    }
    q.st = *reinterpret_cast<const double2 *>(sgt + 2LL * bi);
    if (HAS_S) q.ss = *reinterpret_cast<const double2 *>(sgs + 2LL * bi);
  };

  Regs cur[CPT], nxt[CPT];
#pragma unroll
  for (int r = 0; r < CPT; ++r) {
    cur[r].lk = make_int4(-1, -1, -1, -1);
    nxt[r].lk = make_int4(-1, -1, -1, -1);
  }
  if (compute) {
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      cur[r].lk = load_link(0, r);
      pin_reg(cur[r].lk);
      if (!link_valid(0, r)) cur[r].lk.x = -1;
      load_plane(0, r, cur[r]);
      nxt[r].lk = load_link(min(1, np - 1), r);
    }
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      pin_regs_pair(cur[r]);
      pin_reg(nxt[r].lk);
      if (np < 2 || !link_valid(1, r)) nxt[r].lk.x = -1;
    }
  }

  if (compute) {
    for (int pp = 0; pp < np; ++pp) {
      int4 lk2[CPT];
      const T *rd = lds + (DBUF ? ((pp + 1) & 1) : 0) * 2 * NS * maxp;  // previous plane
      T *wr = lds + (DBUF ? (pp & 1) : 0) * 2 * NS * maxp;
      T res[DBUF ? 1 : CPT][2][NS];  // single buffer: held until every read is done
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        if (r == 0) {
          // the next plane's loads, in flight during this plane's work
#pragma unroll
          for (int r2 = 0; r2 < CPT; ++r2) {
            load_plane(min(pp + 1, np - 1), r2, nxt[r2]);
            lk2[r2] = load_link(min(pp + 2, np - 1), r2);
          }
        }
        const int nbp[3] = {cur[r].lk.y, cur[r].lk.z, cur[r].lk.w};
        // the upwind neighbour's outflow face along d, from slot sl of the
        // neighbouring brick in the previous plane (zero at the boundary)
        auto lds_trace = [&](int d, int sl, T *tr) {
          const int nbit = ((FLIP >> d) & 1) ? 0 : 1;
          const int q = nbp[d] >= 0 ? nbp[d] : 0;
#pragma unroll
          for (int t = 0; t < NS / 2; ++t) {
            const T x = rd[(sl * NS + insert_bit(t, d, nbit)) * maxp + q];  // may be uninitialised: select
            tr[t] = nbp[d] >= 0 ? x : T(0);
          }
        };
        // inflow along d: 4 c on the own inflow face, -2 c on the opposite one
        auto inflow = [&](T *v, int d, const T *tr) {
          const int own0 = (FLIP >> d) & 1;
          const T c4 = T(4) * c[d], c2 = T(2) * c[d];
#pragma unroll
          for (int t = 0; t < NS / 2; ++t) {
            v[insert_bit(t, d, own0)] += c4 * tr[t];
            v[insert_bit(t, d, 1 - own0)] -= c2 * tr[t];
          }
        };
        T v[2][NS];
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int mf = ((PIN || !FX) ? sl : 1 - sl) * NS;
          const int ms = (FX ? 1 - sl : sl) * NS;
          const T sg = T(sl ? cur[r].ss.y : cur[r].ss.x);
#pragma unroll
          for (int b = 0; b < NS; ++b) {
            v[sl][b] = pair_elem<T>(cur[r].f, mf + b);
            if (HAS_S) v[sl][b] += sg * pair_elem<T>(cur[r].s, ms + b);
          }
        }
        T tr[NS / 2], ty[NS / 2], tz[NS / 2];
        lds_trace(0, 1, tr);  // slot 0's x inflow: slot 1 of the x-upwind brick
        inflow(v[0], 0, tr);
        lds_trace(1, 0, tr);
        inflow(v[0], 1, tr);
        lds_trace(2, 0, tr);
        inflow(v[0], 2, tr);
        lds_trace(1, 1, ty);
        lds_trace(2, 1, tz);
        oriented_solve<T, 3, false, FLIP>(v[0], mc, T(cur[r].st.x));
        {
          const int nbit = (FLIP & 1) ? 0 : 1;  // slot 0's outflow face along x
#pragma unroll
          for (int t = 0; t < NS / 2; ++t) tr[t] = v[0][insert_bit(t, 0, nbit)];
        }
        inflow(v[1], 0, tr);
        inflow(v[1], 1, ty);
        inflow(v[1], 2, tz);
        oriented_solve<T, 3, false, FLIP>(v[1], mc, T(cur[r].st.y));
        if (DBUF) {
          if (cur[r].lk.x >= 0) {
#pragma unroll
            for (int sl = 0; sl < 2; ++sl)
#pragma unroll
              for (int b = 0; b < NS; ++b) wr[(sl * NS + b) * maxp + tid + r * tc] = v[sl][b];
            jbuf[(pp & 1) * maxp + tid + r * tc] = (int)base_cell(cur[r].lk.x);
          }
        } else {
#pragma unroll
          for (int sl = 0; sl < 2; ++sl)
#pragma unroll
            for (int b = 0; b < NS; ++b) res[DBUF ? 0 : r][sl][b] = v[sl][b];
        }
      }
      if (!DBUF) {
        lds_barrier();  // every read of the previous plane done
#pragma unroll
        for (int r = 0; r < CPT; ++r)
          if (cur[r].lk.x >= 0) {
#pragma unroll
            for (int sl = 0; sl < 2; ++sl)
#pragma unroll
              for (int b = 0; b < NS; ++b) wr[(sl * NS + b) * maxp + tid + r * tc] = res[DBUF ? 0 : r][sl][b];
            jbuf[tid + r * tc] = (int)base_cell(cur[r].lk.x);
          }
      }
      lds_barrier();  // the plane is complete in LDS
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        pin_regs_pair(nxt[r]);
        pin_reg(lk2[r]);
      }
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        if (pp + 2 >= np || !link_valid(pp + 2, r)) lk2[r].x = -1;
        cur[r] = nxt[r];
        nxt[r].lk = lk2[r];
      }
    }
  } else {
    // store waves: chunk ch (memory order) of CPB bricks per access
    constexpr int CPB = 64 / PQ;
    const int ch = lane / CPB;
    const int m0 = ch * EPC;
    const int sl = (FLIP & 1) ? 1 - m0 / NS : m0 / NS;
    const int b0 = m0 % NS;
    for (int pp = 0; pp < np; ++pp) {
      if (!DBUF) lds_barrier();
      lds_barrier();
      const int n = off[pp + 1] - off[pp];
      const T *pb = lds + (DBUF ? (pp & 1) : 0) * 2 * NS * maxp;
      const int *jb = jbuf + (DBUF ? (pp & 1) : 0) * maxp;
      for (int base = (tid - tc) / 64 * CPB; base < n; base += (NT - tc) / 64 * CPB) {
        const int q = base + lane % CPB;
        if (q < n) {
          T w[EPC];
#pragma unroll
          for (int e = 0; e < EPC; ++e) w[e] = pb[(sl * NS + b0 + e) * maxp + q];
          *reinterpret_cast<float4 *>(uk + (long long)jb[q] * NS + m0) = *reinterpret_cast<float4 *>(w);
        }
      }
    }
  }
}

template <typename T, bool HAS_S, bool DBUF, bool PIN, int CPT, int NT, int MINW>
__global__ __launch_bounds__(NT, MINW) void k_sweep_pair(SweepArgs<T> a, int tc) {
  extern __shared__ __align__(16) unsigned char sweep_smem[];
  T *lds = reinterpret_cast<T *>(sweep_smem);
  constexpr int NB = DBUF ? 2 : 1;
  int *jbuf = reinterpret_cast<int *>(lds + (size_t)NB * 16 * a.bpl.max_plane);
  int *off = jbuf + NB * a.bpl.max_plane;
  for (int i = threadIdx.x; i <= a.bpl.nplanes; i += blockDim.x) off[i] = a.bpl.off[i];
  __syncthreads();
  const int k = blockIdx.x;
  switch (a.ord[k].flip) {
    case 0: sweep_pair_body<T, HAS_S, DBUF, PIN, 0, CPT, NT>(a, k, lds, jbuf, off, tc); break;
    case 1: sweep_pair_body<T, HAS_S, DBUF, PIN, 1, CPT, NT>(a, k, lds, jbuf, off, tc); break;
    case 2: sweep_pair_body<T, HAS_S, DBUF, PIN, 2, CPT, NT>(a, k, lds, jbuf, off, tc); break;
    case 3: sweep_pair_body<T, HAS_S, DBUF, PIN, 3, CPT, NT>(a, k, lds, jbuf, off, tc); break;
    case 4: sweep_pair_body<T, HAS_S, DBUF, PIN, 4, CPT, NT>(a, k, lds, jbuf, off, tc); break;
    case 5: sweep_pair_body<T, HAS_S, DBUF, PIN, 5, CPT, NT>(a, k, lds, jbuf, off, tc); break;
    case 6: sweep_pair_body<T, HAS_S, DBUF, PIN, 6, CPT, NT>(a, k, lds, jbuf, off, tc); break;
    default: sweep_pair_body<T, HAS_S, DBUF, PIN, 7, CPT, NT>(a, k, lds, jbuf, off, tc); break;
  }
}

// Cross sections per orientation in cell-list order (coalesced reads in
// the LDS sweep).
__global__ void k_sigma_planes(const double *__restrict__ sig_t, const double *__restrict__ sig_s, Planes pl,
                               Grid g, double *__restrict__ out) {
  const long long C = g.C;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < 8 * C;
       t += (long long)gridDim.x * blockDim.x) {
    const int flip = (int)(t / C);
    const int idx = (int)(t - flip * C);
    const long long j = flipped_cell(pl.cells[idx], flip, g);
    out[t] = sig_t[j];
    out[8 * C + t] = sig_s[j];
  }
}

// ------------------------------------------------------- coarse Gauss-Seidel
// T_0 has one patch (three ordinates) per octant.  One launch handles one
// diagonal plane of one octant: each (cell, octant) block is solved with
// the patch's own scatter implicit and every other unknown at its latest
// value (Section 5.2).  A cell occupies 2^dim consecutive lanes, one per
// Q1 node; the tensor-product transforms of local_solve.h become lane
// butterflies (__shfl_xor over the node bits), after which lane b holds
// spectral mode b and solves that mode's complex 3x3 system (the three
// ordinates coupled by the self-scatter block) on its own.
//
// Exchanges across the node bits 1, 2 and 4 stay inside 8-lane groups and
// use DPP moves (VALU, no LDS round trip): quad permutations for bits 1
// and 2; for bit 4 the half-row mirror (lane i of 8 takes lane 7 - i)
// followed by the quad reversal (i takes i ^ 3), together i ^ 4.
// (every lane of every row is written, so no prior destination value is
// needed: mov_dpp with bound_ctrl)
__device__ __forceinline__ int dpp_xor(int v, int mask) {
  switch (mask) {
    case 1: return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // quad_perm 1,0,3,2
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);   // quad_perm 2,3,0,1
    case 4: {
      const int t = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror
      return __builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, true);         // quad_perm 3,2,1,0
    }
    default: return __shfl_xor(v, mask, 64);
  }
}

__device__ __forceinline__ double shx(double v, int mask) {
  const long long x = __double_as_longlong(v);
  const int lo = dpp_xor((int)(x & 0xFFFFFFFFLL), mask), hi = dpp_xor((int)(x >> 32), mask);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ cx<double> shx(cx<double> v, int mask) { return {shx(v.re, mask), shx(v.im, mask)}; }

// Node-space 2x2 operator along axis d: out = m_same * own + m_other * partner
// (used for the symmetric mass shapes).
template <int DIM>
__device__ __forceinline__ double lane_mass(double v, int bits_mask, bool inverse) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    if (!((bits_mask >> d) & 1)) continue;
    const double p = shx(v, 1 << d);
    v = inverse ? 4.0 * v - 2.0 * p : (2.0 * v + p) * (1.0 / 6.0);
  }
  return v;
}

template <int DIM>
__device__ __forceinline__ cx<double> lane_forward(double v, int b, const AxisXf<double> *ax) {
  // stage x: real input
  cx<double> y;
  {
    const double p = shx(v, 1);
    const double v0 = (b & 1) ? p : v, v1 = (b & 1) ? v : p;
    cx<double> f0 = ax[0].fwd[0], f1 = ax[0].fwd[1];
    if (b & 1) {
      f0.im = -f0.im;
      f1.im = -f1.im;
    }
    y = cadd(rmul(f0, v0), rmul(f1, v1));
  }
#pragma unroll
  for (int d = 1; d < DIM; ++d) {
    const int bit = 1 << d;
    const cx<double> p = shx(y, bit);
    const cx<double> v0 = (b & bit) ? p : y, v1 = (b & bit) ? y : p;
    cx<double> f0 = ax[d].fwd[0], f1 = ax[d].fwd[1];
    if (b & bit) {
      f0.im = -f0.im;
      f1.im = -f1.im;
    }
    y = cadd(cmul(f0, v0), cmul(f1, v1));
  }
  return y;
}

template <int DIM>
__device__ __forceinline__ double lane_backward(cx<double> U, int b, const AxisXf<double> *ax) {
#pragma unroll
  for (int d = DIM - 1; d >= 0; --d) {
    const int bit = 1 << d;
    const cx<double> p = shx(U, bit);
    const cx<double> u0 = (b & bit) ? p : U, u1 = (b & bit) ? U : p;
    const cx<double> c = (b & bit) ? ax[d].bwd[1] : ax[d].bwd[0];
    const cx<double> cc{c.re, -c.im};
    U = cadd(cmul(c, u0), cmul(cc, u1));
  }
  return U.re;
}

// The same butterflies with each lane's stage coefficients formed once
// (per octant): stage d of the forward transform is y' = A_d y + B_d p with
// p the partner lane's value, and of the inverse U' = C_d U + D_d p; the
// lane's node bit selects which of the axis coefficients (and whether
// their conjugates) A..D are, so the stages themselves take no selects.
struct LaneXf {
  cx<double> fa[3], fb[3], ba[3], bb[3];
};

template <int DIM>
__device__ __forceinline__ LaneXf lane_xf(int flip, bool adj, int b) {
  LaneXf x;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const AxisXf<double> a = axis_xf<double>((flip >> d) & 1, adj);
    const bool hi = (b >> d) & 1;
    const cx<double> f0 = a.fwd[0], f1 = a.fwd[1], c0 = a.bwd[0], c1 = a.bwd[1];
    // forward: bit clear  y' = f0 y + f1 p;  bit set  y' = conj(f1) y + conj(f0) p
    x.fa[d] = hi ? cx<double>{f1.re, -f1.im} : f0;
    x.fb[d] = hi ? cx<double>{f0.re, -f0.im} : f1;
    // inverse: bit clear  U' = c0 U + conj(c0) p;  bit set  U' = conj(c1) U + c1 p
    x.ba[d] = hi ? cx<double>{c1.re, -c1.im} : c0;
    x.bb[d] = hi ? c1 : cx<double>{c0.re, -c0.im};
  }
  return x;
}

template <int DIM>
__device__ __forceinline__ cx<double> lane_forward_x(double v, const LaneXf &x) {
  const double p = shx(v, 1);
  cx<double> y{x.fa[0].re * v + x.fb[0].re * p, x.fa[0].im * v + x.fb[0].im * p};
#pragma unroll
  for (int d = 1; d < DIM; ++d) y = cadd(cmul(x.fa[d], y), cmul(x.fb[d], shx(y, 1 << d)));
  return y;
}

template <int DIM>
__device__ __forceinline__ double lane_backward_x(cx<double> U, const LaneXf &x) {
#pragma unroll
  for (int d = DIM - 1; d >= 1; --d) U = cadd(cmul(x.ba[d], U), cmul(x.bb[d], shx(U, 1 << d)));
  // last stage: only the real part is needed
  const cx<double> p = shx(U, 1);
  return x.ba[0].re * U.re - x.ba[0].im * U.im + x.bb[0].re * p.re - x.bb[0].im * p.im;
}

// What a (cell, octant) update needs that does not depend on earlier
// updates: cell indices, right-hand side and cross sections.  Loaded for
// the next step before the grid barrier that ends the current one.
template <int DIM>
struct GsPrep {
  long long j, jn[DIM];
  double fv[3], st, ss;
  int octant, flip;
  bool has[DIM];
};

template <int DIM, bool ADJ>
__device__ __forceinline__ GsPrep<DIM> gs_prepare(int item, const double *__restrict__ f,
                                                  const double *__restrict__ sig_t, const double *__restrict__ sig_s,
                                                  const OrdInfo *ord_lds, const Planes &pl, const Grid &g, int b) {
  constexpr int NS = 1 << DIM;
  GsPrep<DIM> q;
  q.octant = item >> 28;
  const int idx = item & ((1 << 28) - 1);
  const int k0 = 3 * q.octant;
  q.flip = ord_lds[k0].flip;
  int ci[3], ix[3];
  unpack_cell(pl.cells[idx], q.flip, g, ci, ix);
  q.j = cell_index(ix, g);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int dir = ((q.flip >> d) & 1) ? -1 : 1;
    q.has[d] = ADJ ? (ci[d] < g.n[d] - 1) : (ci[d] > 0);
    int nx[3] = {ix[0], ix[1], ix[2]};
    nx[d] += q.has[d] ? (ADJ ? dir : -dir) : 0;
    q.jn[d] = cell_index(nx, g);
  }
  const long long S = g.S;
#pragma unroll
  for (int m = 0; m < 3; ++m) q.fv[m] = f[(k0 + m) * S + q.j * NS + b];
  q.st = sig_t[q.j];
  q.ss = sig_s[q.j];
  return q;
}

// Accesses of the Gauss-Seidel iterate that are coherent across the XCDs
// without cache maintenance: device-scope relaxed atomics read and write
// at the device coherence point, so a store acknowledged before a flag is
// published is seen by any load issued after the flag is observed.
__device__ __forceinline__ double ld_dev(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Gauss-Seidel update of one (cell, octant) block by the 2^dim lanes of a
// cell group; every lane of the wave must call it (idle groups pass
// active = false with a valid cell and store nothing).  G_lds and ord_lds
// are the level's 24 x 24 scatter block and ordinate data staged in LDS.
// COH: the iterate is read and written with device-coherent accesses.
template <int DIM, bool ADJ, bool COH = false>
__device__ __forceinline__ void gs_update(const GsPrep<DIM> &q, double *__restrict__ u, const double *G_lds,
                                          const OrdInfo *ord_lds, const Grid &g, bool active, int b) {
  constexpr int NS = 1 << DIM;
  const int octant = q.octant, flip = q.flip;
  const int k0 = 3 * octant;
  const long long S = g.S;
  const long long j = q.j;
  const double st = q.st, ss = q.ss;
  const double *up = u + j * NS + b;

  // every value this update reads from earlier updates: all 24 ordinate
  // values at this node and the upwind (adjoint: downwind) traces of the
  // octant's three ordinates
  double uv[24];
#pragma unroll
  for (int kp = 0; kp < 24; ++kp) uv[kp] = COH ? ld_dev(up + kp * S) : up[kp * S];
  double tr[3][DIM];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int fl = (flip >> d) & 1;
      const int nbit = ADJ ? (fl ? 1 : 0) : (fl ? 0 : 1);
      const int bn = (b & ~(1 << d)) | (nbit << d);
      const double *tp = u + (k0 + m) * S + q.jn[d] * NS + bn;
      tr[m][d] = COH ? ld_dev(tp) : *tp;
    }
  }
  // scatter from the other octants' ordinates (latest values)
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int kp = 0; kp < 24; ++kp) {
    const double w = (kp / 3 == octant) ? 0.0 : uv[kp];
#pragma unroll
    for (int m = 0; m < 3; ++m) acc[m] += G_lds[(k0 + m) * 24 + kp] * w;
  }
  double v[3];
  double cc[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const OrdInfo &o = ord_lds[k0 + m];
    cc[m][0] = o.c[0];
    cc[m][1] = o.c[1];
    cc[m][2] = o.c[2];
    if (!ADJ) {
      v[m] = q.fv[m] + ss * acc[m];  // prepared right-hand side f~ = N^{-1} f
    } else {
      v[m] = q.fv[m] + ss * g.vol * lane_mass<DIM>(acc[m], NS - 1, false);
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int fl = (flip >> d) & 1;
      double t = q.has[d] ? tr[m][d] : 0.0;
      if (!ADJ) {
        const int own0 = fl ? 1 : 0;
        v[m] += (((b >> d) & 1) == own0 ? 4.0 : -2.0) * o.c[d] * t;
      } else {
        double hs = 1.0;
#pragma unroll
        for (int e = 0; e < DIM; ++e)
          if (e != d) hs *= g.h[e];
        t = lane_mass<DIM>(t, (NS - 1) & ~(1 << d), false);
        const int own1 = fl ? 0 : 1;
        if (((b >> d) & 1) == own1) v[m] += o.a[d] * hs * t;
      }
    }
  }
  AxisXf<double> ax[3];
#pragma unroll
  for (int d = 0; d < DIM; ++d) ax[d] = axis_xf<double>((flip >> d) & 1, ADJ);
  cx<double> r[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) r[m] = lane_forward<DIM>(v[m], b, ax);
  // this lane's mode: bit d of b selects lambda_- on axis d
  cx<double> M[3][3];
  const double r2 = 1.41421356237309504880;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
#pragma unroll
    for (int mp = 0; mp < 3; ++mp) M[m][mp] = cx<double>{-ss * G_lds[(k0 + m) * 24 + k0 + mp], 0.0};
    double re = st, im = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      re += 2.0 * cc[m][d];
      im += (((b >> d) & 1) ? -r2 : r2) * cc[m][d];
    }
    M[m][m].re += re;
    M[m][m].im += im;
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const cx<double> ip = cinv(M[p][p]);
#pragma unroll
    for (int i = p + 1; i < 3; ++i) {
      const cx<double> l = cmul(M[i][p], ip);
#pragma unroll
      for (int jj = p + 1; jj < 3; ++jj) M[i][jj] = csub(M[i][jj], cmul(l, M[p][jj]));
      r[i] = csub(r[i], cmul(l, r[p]));
    }
  }
#pragma unroll
  for (int p = 2; p >= 0; --p) {
    cx<double> t = r[p];
#pragma unroll
    for (int jj = p + 1; jj < 3; ++jj) t = csub(t, cmul(M[p][jj], r[jj]));
    r[p] = cmul(t, cinv(M[p][p]));
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double out = lane_backward<DIM>(r[m], b, ax);
    if (ADJ) out = lane_mass<DIM>(out, NS - 1, true) * (1.0 / g.vol);
    if (active) {
      if (COH)
        st_dev(u + (k0 + m) * S + j * NS + b, out);
      else
        u[(k0 + m) * S + j * NS + b] = out;
    }
  }
}

// Grid-wide barrier for a cooperative launch without contended atomics:
// every block publishes its arrival generation in its own slot (after a
// release fence that makes its stores visible device-wide), then thread i
// of every block waits for slot i with relaxed loads, followed by one
// acquire fence.  Split in two halves so that independent loads can be
// issued between them.  Spins are bounded; on timeout the error word is set and
// every block leaves its loops, so the kernel always terminates.
struct GridBarrier {
  unsigned *arrive;   // [blocks]
  unsigned *release;  // [1] (unused by the all-to-all form)
  int *err;           // [1]
};

// Arrival half of the barrier: the block's stores are made visible
// device-wide and its slot is set to gen.  A workgroup barrier does not wait
// for other waves' stores to complete, so every wave first waits for its
// own stores (vmcnt(0): acknowledged by the L2); then one thread's release
// fence writes the L2 back and publishes the arrival.
// COH: the data being published were written with device-coherent stores,
// so their acknowledgement is all the release needs (no L2 write-back).
template <bool COH>
__device__ __forceinline__ void grid_arrive(const GridBarrier &gb, unsigned gen) {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), other counters untouched
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!COH) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(gb.arrive + blockIdx.x, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Waiting half: returns false (every thread) after a timeout anywhere.
// COH: the published data are read with device-coherent loads, so no L2
// invalidation is needed after the wait.
template <bool COH>
__device__ __forceinline__ bool grid_wait(const GridBarrier &gb, unsigned gen) {
  __shared__ int ok;
  bool timeout = false;
  for (unsigned i = threadIdx.x; i < gridDim.x; i += blockDim.x) {
    long spins = 0;
    while (__hip_atomic_load(gb.arrive + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
      if (++spins > (1L << 25) || __hip_atomic_load(gb.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(gb.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        timeout = true;
        break;
      }
    }
    if (timeout) break;
  }
  if (!COH && threadIdx.x < gridDim.x) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  if (threadIdx.x == 0) ok = 1;
  __syncthreads();
  if (timeout) ok = 0;
  __syncthreads();
  return ok;
}

// The whole coarse solve (nu sweeps over the octants) as one cooperative
// launch.  The host orders the (sweep, octant, cell) updates into steps:
// an update is placed one step after the latest of its upwind neighbours'
// updates (same sweep and octant) and the same cell's previous update, so
// every value it reads is final and the result equals the sequential
// Gauss-Seidel sweep; items of one step touch distinct cells.  An item is
// (octant << 28) | index into the plane-ordered cell list.  A grid-wide
// barrier separates the steps; the first round of items of the next step
// is prepared before it.
template <int DIM, bool ADJ, int TB, bool COH>
__global__ __launch_bounds__(TB) void k_gs_solve(const double *__restrict__ f, double *__restrict__ u,
                                                  const double *__restrict__ G, const double *__restrict__ sig_t,
                                                  const double *__restrict__ sig_s,
                                                  const OrdInfo *__restrict__ ord, Planes pl, Grid g,
                                                  const int *__restrict__ step_off, const int *__restrict__ items,
                                                  int nsteps, GridBarrier gb, unsigned gen0) {
  constexpr int NS = 1 << DIM;
  constexpr int CPB = TB / NS;  // cells per block per round
  __shared__ double G_lds[24 * 24];
  __shared__ OrdInfo ord_lds[24];
  for (int i = threadIdx.x; i < 24 * 24; i += blockDim.x) G_lds[i] = G[i];
  if (threadIdx.x < 24) ord_lds[threadIdx.x] = ord[threadIdx.x];
  __syncthreads();
  const int b = threadIdx.x & (NS - 1);
  const int slot = threadIdx.x / NS;
  const int stride = gridDim.x * CPB;
  auto first_item = [&](int t, bool &active) {
    const int beg = step_off[t], end = step_off[t + 1];
    const int it = beg + blockIdx.x * CPB + slot;
    active = it < end;
    return items[active ? it : beg];
  };
  bool act;
  GsPrep<DIM> q = gs_prepare<DIM, ADJ>(first_item(0, act), f, sig_t, sig_s, ord_lds, pl, g, b);
  for (int t = 0; t < nsteps; ++t) {
    const int beg = step_off[t], end = step_off[t + 1];
    // the first round was prepared before the barrier; every block runs
    // it so that the wave-wide shuffles see valid lanes
    gs_update<DIM, ADJ, COH>(q, u, G_lds, ord_lds, g, act, b);
    for (int base = beg + blockIdx.x * CPB + stride; base < end; base += stride) {
      const int it = base + slot;
      const bool active = it < end;
      const GsPrep<DIM> q2 =
          gs_prepare<DIM, ADJ>(items[active ? it : beg], f, sig_t, sig_s, ord_lds, pl, g, b);
      gs_update<DIM, ADJ, COH>(q2, u, G_lds, ord_lds, g, active, b);
    }
    // arrive, then load what the next step needs while the other blocks
    // finish (it is read-only data, unaffected by the barrier's fences)
    grid_arrive<COH>(gb, gen0 + t + 1);
    if (t + 1 < nsteps) q = gs_prepare<DIM, ADJ>(first_item(t + 1, act), f, sig_t, sig_s, ord_lds, pl, g, b);
    if (!grid_wait<COH>(gb, gen0 + t + 1)) return;
    asm volatile("" ::: "memory");
  }
}

// Bounded wait of a wave on update counters: each lane with dep >= 0 waits
// for cnt[dep] == c (own = true) or cnt[dep] >= c + 1.  Returns false for
// the whole wave after a timeout anywhere (the error word is set).
__device__ __forceinline__ bool wait_counters(unsigned *cnt, long long dep, unsigned c, bool own, int *err) {
  bool ready = dep < 0;
  long spins = 0;
  bool failed = false;
  while (true) {
    if (!ready) {
      const unsigned v = __hip_atomic_load(cnt + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ready = own ? v == c : v >= c + 1;
    }
    if (__ballot(!ready) == 0) break;
    if (++spins > (1L << 22) ||
        (spins % 64 == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      failed = true;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return __ballot(failed) == 0;
}

// Per-cell pieces of a Gauss-Seidel update shared by the dataflow
// kernels.  gs_cell_setup forms what depends only on the cell's own values
// (the 24 ordinates at the lane's node): the right-hand side without the
// inflow, and the factorised 3 x 3 system of the lane's spectral mode.
// gs_cell_solve adds the inflow traces t (zero where there is no upwind
// neighbour) and solves.
template <int DIM>
struct GsCell {
  double vb[3];
  cx<double> U[3][3], Lf[3][3], dinv[3];
  LaneXf xf;
};

template <int DIM, bool ADJ>
__device__ __forceinline__ void gs_cell_setup(GsCell<DIM> &cs, const double *uv, const double *fv, double st,
                                              double ss, int octant, int b, const double *G_lds,
                                              const OrdInfo *ord_lds, const Grid &g) {
  constexpr int NS = 1 << DIM;
  const int k0 = 3 * octant;
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int kp = 0; kp < 24; ++kp) {
    const double w = (kp / 3 == octant) ? 0.0 : uv[kp];
#pragma unroll
    for (int m = 0; m < 3; ++m) acc[m] += G_lds[(k0 + m) * 24 + kp] * w;
  }
#pragma unroll
  for (int m = 0; m < 3; ++m)
    cs.vb[m] = ADJ ? fv[m] + ss * g.vol * lane_mass<DIM>(acc[m], NS - 1, false) : fv[m] + ss * acc[m];
  // this lane's mode system M = L U (unit L)
  cx<double> (&M)[3][3] = cs.U;
  const double r2 = 1.41421356237309504880;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const OrdInfo &o = ord_lds[k0 + m];
#pragma unroll
    for (int mp = 0; mp < 3; ++mp) M[m][mp] = cx<double>{-ss * G_lds[(k0 + m) * 24 + k0 + mp], 0.0};
    double re = st, im = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      re += 2.0 * o.c[d];
      im += (((b >> d) & 1) ? -r2 : r2) * o.c[d];
    }
    M[m][m].re += re;
    M[m][m].im += im;
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    cs.dinv[p] = cinv(M[p][p]);
#pragma unroll
    for (int i = p + 1; i < 3; ++i) {
      cs.Lf[i][p] = cmul(M[i][p], cs.dinv[p]);
#pragma unroll
      for (int jj = p + 1; jj < 3; ++jj) M[i][jj] = csub(M[i][jj], cmul(cs.Lf[i][p], M[p][jj]));
    }
  }
  cs.xf = lane_xf<DIM>(ord_lds[k0].flip, ADJ, b);
}

template <int DIM, bool ADJ>
__device__ __forceinline__ void gs_cell_solve(const GsCell<DIM> &cs, const double (&t)[3][DIM], int octant,
                                              int flip, int b, const OrdInfo *ord_lds, const Grid &g,
                                              double *out) {
  constexpr int NS = 1 << DIM;
  const int k0 = 3 * octant;
  double v[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const OrdInfo &o = ord_lds[k0 + m];
    v[m] = cs.vb[m];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int fl = (flip >> d) & 1;
      if (!ADJ) {
        const int own0 = fl ? 1 : 0;
        v[m] += (((b >> d) & 1) == own0 ? 4.0 : -2.0) * o.c[d] * t[m][d];
      } else {
        double hs = 1.0;
#pragma unroll
        for (int e = 0; e < DIM; ++e)
          if (e != d) hs *= g.h[e];
        const double tm = lane_mass<DIM>(t[m][d], (NS - 1) & ~(1 << d), false);
        const int own1 = fl ? 0 : 1;
        if (((b >> d) & 1) == own1) v[m] += o.a[d] * hs * tm;
      }
    }
  }
  cx<double> r[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) r[m] = lane_forward_x<DIM>(v[m], cs.xf);
#pragma unroll
  for (int i = 1; i < 3; ++i)
#pragma unroll
    for (int q = 0; q < i; ++q) r[i] = csub(r[i], cmul(cs.Lf[i][q], r[q]));
#pragma unroll
  for (int q = 2; q >= 0; --q) {
    cx<double> x = r[q];
#pragma unroll
    for (int jj = q + 1; jj < 3; ++jj) x = csub(x, cmul(cs.U[q][jj], r[jj]));
    r[q] = cmul(x, cs.dinv[q]);
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double o = lane_backward_x<DIM>(r[m], cs.xf);
    if (ADJ) o = lane_mass<DIM>(o, NS - 1, true) * (1.0 / g.vol);
    out[m] = o;
  }
}

// Dataflow form of the same coarse solve: no grid-wide barrier.  Every
// cell j has a counter cnt[j] of completed updates; the update with count
// c = 8 sweep + (octant's position in the order) may run once cnt[j] == c
// (the cell's earlier updates are done) and cnt[n] >= c + 1 for each upwind
// (adjoint: downwind) neighbour n (its update of the same sweep and octant
// is done).  That is exactly the data each update reads; writes it could
// race with are excluded too, since a neighbour cannot reach its next update
// of this octant before this cell has passed the reflected octant, which
// comes later in this cell's chain.  Each wave runs a list of slots of 8
// updates (one per 2^dim-lane group) in step order of the pipelined
// schedule, so the earliest unfinished step always has all its updates
// runnable and the launch cannot deadlock (every wave is resident: it is a
// cooperative launch).  Publishing: the wave's stores are released at
// device scope (device-coherent stores, waited for), then each group's
// leader stores c + 1 in cnt[j]; waiting: relaxed polls of the counters,
// after which the iterate is read with device-coherent loads.  The wait is
// in two parts: the cell's own counter first, after which the scatter from
// the other octants and the factorised mode systems are formed, then the
// neighbours' counters and the inflow traces.  Spins are bounded and set
// the error word, which every waiting wave checks.
// Slot items: octant << 29 | c << 22 | cell-list index (all ones: empty;
// c <= 126 for real items).
template <int DIM, bool ADJ>
__global__ __launch_bounds__(256) void k_gs_flow(const double *__restrict__ f, double *u,
                                                 const double *__restrict__ G, const double *__restrict__ sig_t,
                                                 const double *__restrict__ sig_s,
                                                 const OrdInfo *__restrict__ ord, Planes pl, Grid g,
                                                 const int *__restrict__ wave_off, const int *__restrict__ slots,
                                                 int nwaves, unsigned *cnt, int *err) {
  constexpr int NS = 1 << DIM;
  __shared__ double G_lds[24 * 24];
  __shared__ OrdInfo ord_lds[24];
  for (int i = threadIdx.x; i < 24 * 24; i += blockDim.x) G_lds[i] = G[i];
  if (threadIdx.x < 24) ord_lds[threadIdx.x] = ord[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int b = lane & (NS - 1);
  const int grp = lane / NS;  // 64 / 2^dim groups per wave (8 in 3-D)
  const int wave = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (wave >= nwaves) return;
  const long long S = g.S;
  const int s0 = wave_off[wave], s1 = wave_off[wave + 1];
  for (int sl = s0; sl < s1; ++sl) {
    const int item = slots[(long long)sl * (64 / NS) + grp];
    const bool active = item != -1;  // all ones: c = 127 never occurs
    const int octant = active ? (item >> 29) & 7 : 0;
    const unsigned c = active ? (unsigned)((item >> 22) & 127) : 0u;
    const int idx = active ? item & ((1 << 22) - 1) : 0;
    const int k0 = 3 * octant;
    // read-only data of the update first (overlapping the waits)
    const GsPrep<DIM> q = gs_prepare<DIM, ADJ>((octant << 28) | idx, f, sig_t, sig_s, ord_lds, pl, g, b);
    const long long jself = q.j;
    // wait for the cell's own earlier updates (lane 0 of each group) while
    // lane 1 + d samples the upwind (adjoint: downwind) neighbour along
    // axis d in the same round trips.  If the neighbours are all done the
    // iterate and the inflow traces are fetched together; otherwise the
    // set-up that needs only the own values is formed first, then the
    // neighbours are awaited.
    long long dep = -1;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      if (active && q.has[d] && b == 1 + d) dep = q.jn[d];
    bool up_ready;
    {
      const bool own = active && b == 0;
      bool ready = !own, upr = dep < 0;
      long spins = 0;
      bool failed = false;
      while (true) {
        if (!ready) ready = __hip_atomic_load(cnt + jself, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == c;
        if (!upr) upr = __hip_atomic_load(cnt + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= c + 1;
        if (__ballot(!ready) == 0) break;
        if (++spins > (1L << 22) ||
            (spins % 64 == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          failed = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (__ballot(failed) != 0) return;
      up_ready = __ballot(!upr) == 0;
    }
    asm volatile("" ::: "memory");
    const double *up = u + jself * NS + b;
    double uv[24];
#pragma unroll
    for (int kp = 0; kp < 24; ++kp) uv[kp] = ld_dev(up + kp * S);
    double t[3][DIM];
    auto load_traces = [&]() {
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const int fl = (q.flip >> d) & 1;
          const int nbit = ADJ ? (fl ? 1 : 0) : (fl ? 0 : 1);
          const int bn = (b & ~(1 << d)) | (nbit << d);
          t[m][d] = q.has[d] ? ld_dev(u + (k0 + m) * S + q.jn[d] * NS + bn) : 0.0;
        }
    };
    if (up_ready) load_traces();
    GsCell<DIM> cs;
    gs_cell_setup<DIM, ADJ>(cs, uv, q.fv, q.st, q.ss, octant, b, G_lds, ord_lds, g);
    if (!up_ready) {
      if (!wait_counters(cnt, dep, c, false, err)) return;
      asm volatile("" ::: "memory");
      load_traces();
    }
    double out[3];
    gs_cell_solve<DIM, ADJ>(cs, t, octant, q.flip, b, ord_lds, g, out);
    if (active)
#pragma unroll
      for (int m = 0; m < 3; ++m) st_dev(u + (k0 + m) * S + jself * NS + b, out[m]);
    // the group's iterate stores are acknowledged at the device coherence
    // point before its counter moves
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    asm volatile("" ::: "memory");
    if (active && b == 0) __hip_atomic_store(cnt + jself, c + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Brick form of the dataflow solve (3-D, even cell counts): one
// workgroup of three waves updates a 2 x 2 x 2 brick of cells for one
// (sweep, octant); wave m takes ordinate 3 octant + m of the octant's patch
// at the brick's 64 cell nodes (8 lanes per cell).  Dependencies and
// counters are per brick (cnt[B] = updates done), so fewer dependent steps
// cross the device than in the cell form (the brick grid is half as wide).
// Inside the brick the cells are taken in the four diagonal planes of the
// sweep direction; the inflow a cell takes from a neighbour in the same
// brick comes from that cell's lanes by a shuffle, from a neighbour
// outside it by a device-coherent load.  Per plane each wave transforms
// its own ordinate only; the 3 x 3 mode coupling is a product with the
// lane's row of the inverse mode matrix (formed in the set-up, off the
// dependent chain) after the three waves exchange their transformed
// right-hand sides through LDS (one barrier per plane).
// Slot items: octant << 29 | c << 22 | brick index (one brick per slot);
// one workgroup of 192 threads per slot list.
template <bool ADJ>
__global__ __launch_bounds__(192) void k_gs_brick(const double *__restrict__ f, double *u,
                                                   const double *__restrict__ G, const double *__restrict__ sig_t,
                                                   const double *__restrict__ sig_s,
                                                   const OrdInfo *__restrict__ ord, Grid g,
                                                   const int *__restrict__ wave_off, const int *__restrict__ slots,
                                                   int nlists, unsigned *cnt, int *err) {
  constexpr int DIM = 3, NS = 8;
  __shared__ double G_lds[24 * 24];
  __shared__ OrdInfo ord_lds[24];
  __shared__ cx<double> rx[2][3][64];  // transformed right-hand sides, by plane parity
  __shared__ int up_flag;               // wave 0 found the upwind bricks done
  for (int i = threadIdx.x; i < 24 * 24; i += blockDim.x) G_lds[i] = G[i];
  if (threadIdx.x < 24) ord_lds[threadIdx.x] = ord[threadIdx.x];
  __syncthreads();
  const int list = blockIdx.x;
  if (list >= nlists) return;  // uniform over the workgroup
  const int lane = threadIdx.x & 63;
  const int m = threadIdx.x >> 6;  // ordinate of the patch (wave-uniform)
  const int m1 = m == 0 ? 1 : 0, m2 = m == 2 ? 1 : 2;  // the other two
  const int b = lane & 7;
  const int grp = lane >> 3;
  const int sub = (grp & 1) + ((grp >> 1) & 1) + ((grp >> 2) & 1);
  const int nb[3] = {g.n[0] / 2, g.n[1] / 2, g.n[2] / 2};
  const long long S = g.S;
  const double r2 = 1.41421356237309504880;
  const int s0 = wave_off[list], s1 = wave_off[list + 1];
  for (int sl = s0; sl < s1; ++sl) {
    const int item = __builtin_amdgcn_readfirstlane(slots[sl]);
    const int octant = (item >> 29) & 7;
    const unsigned c = (unsigned)((item >> 22) & 127);
    const int B = item & ((1 << 22) - 1);
    const int k0 = 3 * octant;
    const int km = k0 + m;
    const int flip = ord_lds[k0].flip;
    const int bx[3] = {B % nb[0], (B / nb[0]) % nb[1], B / (nb[0] * nb[1])};
    int ix[3], nbr[3];
    long long jn[3];
    bool ext[3];
    long long mydep = -1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const bool rev = (((flip >> d) & 1) != 0) != ADJ;  // sweep runs towards lower indices
      const int pb = rev ? nb[d] - 1 - bx[d] : bx[d];
      const int lp = (grp >> d) & 1;
      const int pc = 2 * pb + lp;
      ix[d] = rev ? g.n[d] - 1 - pc : pc;
      ext[d] = lp == 0 && pc > 0;
      nbr[d] = rev ? ix[d] + 1 : ix[d] - 1;
      if (grp == 0 && b == 1 + d && pb > 0) {
        int by[3] = {bx[0], bx[1], bx[2]};
        by[d] += rev ? 1 : -1;
        mydep = by[0] + (long long)nb[0] * (by[1] + (long long)nb[1] * by[2]);
      }
    }
    if (lane == 0) mydep = B;
    const long long j = cell_index(ix, g);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int nx[3] = {ix[0], ix[1], ix[2]};
      nx[d] = ext[d] ? nbr[d] : ix[d];
      jn[d] = cell_index(nx, g);
    }
    const double fv = f[km * S + j * NS + b];
    const double st = sig_t[j], ss = sig_s[j];

    // Waits are taken by wave 0 alone and passed on through the barrier,
    // so the three waves leave together.  Lane 0 polls the brick's own
    // earlier update; lanes 1..3 sample the upwind bricks in the same
    // round trips.  When these are already done, the iterate and the
    // inflow traces are fetched at once; otherwise the set-up is formed
    // first and wave 0 then waits for the upwind bricks.
    bool ok = true, up_ready = true;
    if (m == 0) {
      const bool own = lane == 0;
      bool ready = !own, upr = mydep < 0 || own;
      long spins = 0;
      while (true) {
        if (!ready) ready = __hip_atomic_load(cnt + mydep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == c;
        if (!upr) upr = __hip_atomic_load(cnt + mydep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= c + 1;
        if (__ballot(!ready) == 0) break;
        if (++spins > (1L << 22) ||
            (spins % 64 == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      up_ready = __ballot(!upr) == 0;
      if (lane == 0) up_flag = up_ready ? 1 : 0;
    }
    if (__syncthreads_or(!ok)) return;  // a wait timed out (err is set)
    up_ready = up_flag != 0;
    asm volatile("" ::: "memory");
    double uv[24];
    {
      const double *up = u + j * NS + b;
#pragma unroll
      for (int kp = 0; kp < 24; ++kp) uv[kp] = ld_dev(up + kp * S);
    }
    double tex[DIM] = {0.0, 0.0, 0.0};
    if (up_ready) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int nbit = (((flip >> d) & 1) != 0) == ADJ ? 1 : 0;  // the upwind cell's outflow node
        const int bn = (b & ~(1 << d)) | (nbit << d);
        tex[d] = ext[d] ? ld_dev(u + km * S + jn[d] * NS + bn) : 0.0;
      }
    }
    double acc = 0.0;
#pragma unroll
    for (int kp = 0; kp < 24; ++kp) acc += (kp / 3 == octant) ? 0.0 : G_lds[km * 24 + kp] * uv[kp];
    const double vb = ADJ ? fv + ss * g.vol * lane_mass<DIM>(acc, NS - 1, false) : fv + ss * acc;
    // mode matrix M = L U (unit L) of the three ordinates at mode b
    cx<double> M[3][3], Lf[3][3], dinv[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const OrdInfo &o = ord_lds[k0 + q];
#pragma unroll
      for (int qp = 0; qp < 3; ++qp) M[q][qp] = cx<double>{-ss * G_lds[(k0 + q) * 24 + k0 + qp], 0.0};
      double re = st, im = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        re += 2.0 * o.c[d];
        im += (((b >> d) & 1) ? -r2 : r2) * o.c[d];
      }
      M[q][q].re += re;
      M[q][q].im += im;
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      dinv[p] = cinv(M[p][p]);
#pragma unroll
      for (int i = p + 1; i < 3; ++i) {
        Lf[i][p] = cmul(M[i][p], dinv[p]);
#pragma unroll
        for (int jj = p + 1; jj < 3; ++jj) M[i][jj] = csub(M[i][jj], cmul(Lf[i][p], M[p][jj]));
      }
    }
    // row m of M^-1 solves M^T y = e_m:  U^T z = e_m, then L^T y = z
    cx<double> w[3], z[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      cx<double> s{q == m ? 1.0 : 0.0, 0.0};
#pragma unroll
      for (int qq = 0; qq < q; ++qq) s = csub(s, cmul(M[qq][q], z[qq]));
      z[q] = cmul(s, dinv[q]);
    }
#pragma unroll
    for (int q = 2; q >= 0; --q) {
      cx<double> s = z[q];
#pragma unroll
      for (int qq = q + 1; qq < 3; ++qq) s = csub(s, cmul(Lf[qq][q], w[qq]));
      w[q] = s;
    }
    const LaneXf xf = lane_xf<DIM>(flip, ADJ, b);
    if (!up_ready) {
      if (m == 0) ok = wait_counters(cnt, lane != 0 ? mydep : -1, c, false, err);
      if (__syncthreads_or(!ok)) return;
      asm volatile("" ::: "memory");
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int nbit = (((flip >> d) & 1) != 0) == ADJ ? 1 : 0;  // the upwind cell's outflow node
        const int bn = (b & ~(1 << d)) | (nbit << d);
        tex[d] = ext[d] ? ld_dev(u + km * S + jn[d] * NS + bn) : 0.0;
      }
    }

    const OrdInfo &om = ord_lds[km];
    // the row's entries for this wave's ordinate and the other two
    // (selects: m is uniform but not a compile-time index)
    const cx<double> wm = m == 0 ? w[0] : (m == 1 ? w[1] : w[2]);
    const cx<double> wm1 = m == 0 ? w[1] : w[0];
    const cx<double> wm2 = m == 2 ? w[1] : w[2];
    double res = 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      double v = vb;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int fl = (flip >> d) & 1;
        const int nbit = (fl != 0) == ADJ ? 1 : 0;
        const int bn = (b & ~(1 << d)) | (nbit << d);
        // the upwind cell inside the brick finished in the previous plane
        const double tin = __shfl(res, ((grp ^ (1 << d)) << 3) | bn, 64);
        const double t = ((grp >> d) & 1) ? tin : tex[d];
        if (!ADJ) {
          v += (((b >> d) & 1) == fl ? 4.0 : -2.0) * om.c[d] * t;
        } else {
          // adjoint: the face mass on the other axes, on the lane's own face side
          double hs = 1.0;
#pragma unroll
          for (int e = 0; e < DIM; ++e)
            if (e != d) hs *= g.h[e];
          const double tm = lane_mass<DIM>(t, (NS - 1) & ~(1 << d), false);
          if (((b >> d) & 1) == (fl ? 0 : 1)) v += om.a[d] * hs * tm;
        }
      }
      const cx<double> r = lane_forward_x<DIM>(v, xf);
      rx[p & 1][m][lane] = r;
      __syncthreads();
      const cx<double> x = cadd(cadd(cmul(wm, r), cmul(wm1, rx[p & 1][m1][lane])), cmul(wm2, rx[p & 1][m2][lane]));
      double o = lane_backward_x<DIM>(x, xf);
      if (ADJ) o = lane_mass<DIM>(o, NS - 1, true) * (1.0 / g.vol);
      if (sub == p) res = o;
    }
    st_dev(u + km * S + j * NS + b, res);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's stores are acknowledged
    asm volatile("" ::: "memory");
    __syncthreads();                     // ... and those of the other two waves
    if (threadIdx.x == 0) __hip_atomic_store(cnt + B, c + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------- conversions
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_convert(const Tin *__restrict__ in, Tout *__restrict__ out, int P,
                                                    long long S, const double *__restrict__ pre,
                                                    const double *__restrict__ post, double scale,
                                                    double *__restrict__ out64) {
  // one thread per (patch, spatial dof), 32-bit indices (below 2^32,
  // checked at launch)
  const unsigned t = blockIdx.x * (unsigned)kBlock + threadIdx.x;
  if (t < (unsigned)P * (unsigned)S) {
    const unsigned p = t / (unsigned)S;
    const long long s = t - p * (unsigned)S;
    double x[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      x[m] = (double)in[(3LL * p + m) * S + s] * scale;
      if (pre) x[m] *= pre[3 * p + m];
    }
    const double sum = x[0] + x[1] + x[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double y = 2.0 * x[k] - sum * (1.0 / 3.0);   // Psi^{-1} = 2 I - J / 3
      if (post) y *= post[3 * p + k];
      const Tout yo = (Tout)y;
      out[(3LL * p + k) * S + s] = yo;
      // the same values widened (a second copy in FP64, from the rounded ones)
      if (out64) out64[(3LL * p + k) * S + s] = (double)yo;
    }
  }
}

// Conversion of a forward right-hand side into prepared ordinate form:
// the ordinate conversion above, then the inverse cell mass matrix applied
// per ordinate (f~ = N^{-1} f).  One lane per (patch, spatial dof): the
// 2^dim lanes of a cell are one aligned group and the inverse mass shape is
// a lane exchange inside it; reads and writes of consecutive lanes are
// consecutive (plane layout: whole cells at their list positions).
template <typename Tin, typename Tout, int DIM>
__global__ __launch_bounds__(kBlock) void k_convert_minv(const Tin *__restrict__ in, Tout *__restrict__ out, int P,
                                                         Grid g, const double *__restrict__ pre,
                                                         const double *__restrict__ post,
                                                         const int *__restrict__ pos,
                                                         const OrdInfo *__restrict__ ord, double scale) {
  constexpr int NS = 1 << DIM;
  const unsigned S = (unsigned)g.S;
  const unsigned t = blockIdx.x * (unsigned)kBlock + threadIdx.x;
  if (t >= (unsigned)P * S) return;  // whole cell groups
  const unsigned p = t / S;
  const unsigned rem = t - p * S;
  const unsigned j = rem >> DIM;
  const double iv = 1.0 / g.vol;
  double x[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) x[m] = (double)in[(3LL * p + m) * S + rem] * ((pre ? pre[3 * p + m] : 1.0) * scale);
  // plane layout (the three ordinates of a patch share the orientation)
  const unsigned jo = pos ? (unsigned)pos[(long long)ord[3 * p].flip * g.C + j] : j;
  const long long ro = ((long long)jo << DIM) + (rem & (NS - 1));
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double y = (2.0 * x[k] - (x[0] + x[1] + x[2]) * (1.0 / 3.0)) * (post ? post[3 * p + k] : 1.0);
    out[(3LL * p + k) * S + ro] = (Tout)(lane_mass<DIM>(y, NS - 1, true) * iv);
  }
}

// ------------------------------------------------------------- transfers
template <typename Tin, typename Tout, int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict(const Tin *__restrict__ s_new, const Tin *__restrict__ s_prev,
                                                     Tout *__restrict__ fc, const double *__restrict__ R,
                                                     const int *__restrict__ first_child,
                                                     const int *__restrict__ n_child, int Pc,
                                                     const double *__restrict__ sig_s, int apply_sn, Grid g,
                                                     const int *__restrict__ pos, const OrdInfo *__restrict__ cord) {
  // one lane per (coarse patch, spatial dof): consecutive lanes read and
  // write consecutive values, the 2^dim lanes of a cell are one aligned
  // group (the mass shape of the adjoint is a lane exchange inside it)
  constexpr int NS = 1 << DIM;
  const unsigned S = (unsigned)g.S;
  const unsigned t = blockIdx.x * (unsigned)kBlock + threadIdx.x;
  if (t >= (unsigned)Pc * S) return;  // whole cell groups (S is a multiple of 2^dim)
  const unsigned p = t / S;
  const unsigned rem = t - p * S;
  const unsigned j = rem >> DIM;
  const int c0 = first_child[p], nc = n_child[p];
  const double fsn = apply_sn ? sig_s[j] * g.vol : 1.0;
  double out[3] = {0.0, 0.0, 0.0};
  for (int cb = 0; cb < nc; cb += 4) {
    // the loads of up to four children first (a parent has one or four)
    Tin xr[4][3];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      const unsigned c = (unsigned)(c0 + min(cb + cc, nc - 1));
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const long long off = (3LL * c + m) * S + rem;
        Tin v = s_new[off];
        if (s_prev) v -= s_prev[off];
        xr[cc][m] = v;
      }
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      if (cb + cc >= nc) break;
      const double *Rc = R + 9LL * (c0 + cb + cc);
      double x[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        x[m] = (double)xr[cc][m];
        if (apply_sn) x[m] = fsn * lane_mass<DIM>(x[m], NS - 1, false);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) out[k] += Rc[k * 3] * x[0] + Rc[k * 3 + 1] * x[1] + Rc[k * 3 + 2] * x[2];
    }
  }
  // plane layout: the cell's position in its ordinate's sweep list (the
  // three ordinates of a patch share the orientation)
  const unsigned jo = pos ? (unsigned)pos[(long long)cord[3 * p].flip * g.C + j] : j;
#pragma unroll
  for (int k = 0; k < 3; ++k) fc[(3LL * p + k) * S + ((long long)jo << DIM) + (rem & (NS - 1))] = (Tout)out[k];
}

// One thread per (coarse patch p, spatial dof s): the parent's three values
// are read once for all of its children (one, or four when it is refined),
// whose fine values are then written (added to with add).
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_prolong(const Tin *__restrict__ uc, Tout *__restrict__ uf,
                                                    const double *__restrict__ Pb,
                                                    const int *__restrict__ first_child,
                                                    const int *__restrict__ n_child, int Pc, long long S, int add) {
  // 32-bit indices (patches x spatial dofs < 2^32, checked at launch)
  const unsigned t = blockIdx.x * (unsigned)kBlock + threadIdx.x;
  if (t < (unsigned)Pc * (unsigned)S) {
    const unsigned p = t / (unsigned)S;
    const long long s = t - p * (unsigned)S;
    double x[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = (double)uc[(3LL * p + d) * S + s];
    const int c0 = first_child[p], nc = n_child[p];
    Tout f[4][3];
    if (add) {
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int c = c0 + min(cc, nc - 1);
#pragma unroll
        for (int k = 0; k < 3; ++k) f[cc][k] = uf[(3LL * c + k) * S + s];
      }
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      if (cc >= nc) break;
      const int c = c0 + cc;
      const double *B = Pb + 9LL * c;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double y = B[k * 3] * x[0] + B[k * 3 + 1] * x[1] + B[k * 3 + 2] * x[2];
        if (add) y += (double)f[cc][k];
        uf[(3LL * c + k) * S + s] = (Tout)y;
      }
    }
  }
}

// --------------------------------------------------------- operator apply
// Apply 2x2 matrix [[m00, m01], [m10, m11]] along axis d (physical order).
template <int DIM>
__device__ __forceinline__ void axis_apply(double *v, int d, double m00, double m01, double m10, double m11) {
  constexpr int NS = 1 << DIM;
  const int bit = 1 << d;
#pragma unroll
  for (int b = 0; b < NS; ++b) {
    if (b & bit) continue;
    const double p0 = v[b], p1 = v[b | bit];
    v[b] = m00 * p0 + m01 * p1;
    v[b | bit] = m10 * p0 + m11 * p1;
  }
}

// y = L x - sigma_s N (S~ x) on the finest level, canonical layout.
// Forward:  per patch, u = Psi x, per ordinate r_k = A_loc u_k - upwind
//           coupling, y = Psi W r.
// Adjoint:  L^T = Psi L^T_ord W Psi: mu = W Psi x, r_k = A_loc^T mu_k -
//           downwind coupling, y = Psi r (S is symmetric, so S^T x = S x).
template <int DIM, bool ADJ, typename TX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_apply_cells(const TX *__restrict__ x, const double *__restrict__ s,
                                                        double *__restrict__ y, const double *__restrict__ sig_t,
                                                        const double *__restrict__ sig_s,
                                                        const OrdInfo *__restrict__ ord, const double *__restrict__ w,
                                                        int P, Grid g, int per_xcd) {
  constexpr int NS = 1 << DIM;
  constexpr double m6 = 1.0 / 6.0;
  // one (patch, cell) per thread; the workgroups of one XCD (dispatched
  // round-robin over the 8) take one contiguous run of cells, so the
  // neighbour cells one row or plane back are read from the same L2
  const long long lb = (long long)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  const long long t = lb * kBlock + threadIdx.x;
  const long long C = g.C, S = g.S;
  if (t >= (long long)P * C) return;
  // 32-bit index arithmetic (patches x cells < 2^31, checked at launch)
  const unsigned tt = (unsigned)t;
  const unsigned q = tt / (unsigned)C;
  const unsigned ju = tt - q * (unsigned)C;
  const unsigned r0 = ju / (unsigned)g.n[0];
  const int ix[3] = {(int)(ju - r0 * (unsigned)g.n[0]), (int)(r0 % (unsigned)g.n[1]), (int)(r0 / (unsigned)g.n[1])};
  const long long j = ju;
  const int fl0 = ord[3 * q].flip;  // the three ordinates of a patch share the octant
  auto vec_load = [&](const double *p, double *v) {
#pragma unroll
    for (int b = 0; b < NS; b += 2) {
      const double2 u = *reinterpret_cast<const double2 *>(p + b);
      v[b] = u.x;
      v[b + 1] = u.y;
    }
  };
  // x in FP64, or FP32 widened exactly
  auto x_load = [&](const TX *p, double *v) {
    if constexpr (sizeof(TX) == 8) {
      vec_load(reinterpret_cast<const double *>(p), v);
    } else {
#pragma unroll
      for (int b = 0; b < NS; b += 4) {
        const float4 u = *reinterpret_cast<const float4 *>(p + b);
        v[b] = u.x;
        v[b + 1] = u.y;
        v[b + 2] = u.z;
        v[b + 3] = u.w;
      }
    }
  };
  double xv[3][NS];
#pragma unroll
  for (int m = 0; m < 3; ++m) x_load(x + (3LL * q + m) * S + j * NS, xv[m]);
  double hs[3];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    hs[d] = 1.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e)
      if (e != d) hs[d] *= g.h[e];
  }
  // T1 along d oriented with the flow (its transpose for the adjoint)
  auto stream_axis = [&](double *v, int d) {
    if (((fl0 >> d) & 1) != (ADJ ? 1 : 0))
      axis_apply<DIM>(v, d, 0.5, -0.5, 0.5, 0.5);
    else
      axis_apply<DIM>(v, d, 0.5, 0.5, -0.5, 0.5);
  };
  auto mass_axis = [&](double *v, int d) { axis_apply<DIM>(v, d, 2.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 2.0 / 6.0); };
  // volume terms of every ordinate: r_k = sigma_t vol N u_k + sum_d c_kd
  // T1_d (x) N on the other axes u_k, the axis products shared between
  // the terms (3-D: 7 axis products instead of 12, 2-D: 5 instead of 6)
  const double stv = sig_t[j] * g.vol;
  double yk[3][NS];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const OrdInfo &o = ord[3 * q + k];
    const double wk = ADJ ? w[3 * q + k] : 1.0;
    const double wo = ADJ ? 1.0 : w[3 * q + k];
    double c[3];
#pragma unroll
    for (int d = 0; d < DIM; ++d) c[d] = o.a[d] * hs[d];
    double u[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) u[b] = wk * (xv[0][b] + xv[1][b] + xv[2][b] + 3.0 * xv[k][b]) * m6;
    // e, c and u are overwritten in place (three arrays live)
    double e[NS], c1[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) e[b] = u[b];
    if constexpr (DIM == 3) {
      stream_axis(e, 2);
      mass_axis(e, 1);  // e = N_y T_z u
      mass_axis(u, 2);  // u = N_z u
#pragma unroll
      for (int b = 0; b < NS; ++b) c1[b] = u[b];
      stream_axis(c1, 1);  // c1 = T_y N_z u
      mass_axis(u, 1);     // u = N_y N_z u
#pragma unroll
      for (int b = 0; b < NS; ++b) c1[b] = stv * u[b] + c[1] * c1[b] + c[2] * e[b];
      mass_axis(c1, 0);    // N_x (sigma_t vol N_y N_z u + c_y T_y N_z u + c_z N_y T_z u)
      stream_axis(u, 0);   // u = T_x N_y N_z u
    } else {
      mass_axis(e, 0);
      stream_axis(e, 1);  // e = T_y N_x u
      mass_axis(u, 1);    // u = N_y u
#pragma unroll
      for (int b = 0; b < NS; ++b) c1[b] = u[b];
      mass_axis(c1, 0);  // c1 = N_x N_y u
#pragma unroll
      for (int b = 0; b < NS; ++b) c1[b] = stv * c1[b] + c[1] * e[b];
      stream_axis(u, 0);  // u = T_x N_y u
    }
    double r[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) r[b] = c1[b] + c[0] * u[b];
#pragma unroll
    for (int b = 0; b < NS; ++b) yk[k][b] = wo * r[b];
  }
  // minus the coupling to the upwind (adjoint: downwind) neighbour along
  // each axis: the neighbour's opposite face, applied on the own face
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int fl = (fl0 >> d) & 1;
    const int step = (fl ? 1 : -1) * (ADJ ? -1 : 1);
    const bool has = step > 0 ? (ix[d] < g.n[d] - 1) : (ix[d] > 0);
    if (!has) continue;
    const long long jn = j + (d == 0 ? step : d == 1 ? step * (long long)g.n[0] : step * (long long)g.n[0] * g.n[1]);
    const int nbit = (fl ? 0 : 1) ^ (ADJ ? 1 : 0);
    const int own = 1 - nbit;
    double xf[3][NS / 2];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const TX *pn = x + (3LL * q + m) * S + jn * NS;
#pragma unroll
      for (int u = 0; u < NS / 2; ++u) xf[m][u] = (double)pn[insert_bit(u, d, nbit)];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const OrdInfo &o = ord[3 * q + k];
      const double wk = ADJ ? w[3 * q + k] : 1.0;
      const double wo = ADJ ? 1.0 : w[3 * q + k];
      double tr[NS / 2];
#pragma unroll
      for (int u = 0; u < NS / 2; ++u) tr[u] = wk * (xf[0][u] + xf[1][u] + xf[2][u] + 3.0 * xf[k][u]) * m6;
      mass_shape<double, DIM - 1, false>(tr);
      const double cn = wo * o.a[d] * hs[d];
      // node b takes face value b without bit d, on the own face only
      // (compile-time register indices: a selected factor, not a select of
      // the register)
#pragma unroll
      for (int b = 0; b < NS; ++b) {
        const int u = (b & ((1 << d) - 1)) | ((b >> (d + 1)) << d);
        yk[k][b] -= (((b >> d) & 1) == own ? cn : 0.0) * tr[u];
      }
    }
  }
  const double ssv = sig_s[j] * g.vol;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double sv[NS];
    vec_load(s + (3LL * q + m) * S + j * NS, sv);
    mass_shape<double, DIM, false>(sv);
    double out[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) out[b] = (yk[0][b] + yk[1][b] + yk[2][b] + 3.0 * yk[m][b]) * m6 - ssv * sv[b];
    double *po = y + (3LL * q + m) * S + j * NS;
#pragma unroll
    for (int b = 0; b < NS; b += 2) *reinterpret_cast<double2 *>(po + b) = make_double2(out[b], out[b + 1]);
  }
}

template <typename T, int DIM>
__global__ void k_scale_sn(const T *__restrict__ in, T *__restrict__ out, const double *__restrict__ sig_s, int A,
                           Grid g) {
  constexpr int NS = 1 << DIM;
  const long long total = (long long)A * g.C;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long j = t % g.C;
    double v[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) v[b] = (double)in[t * NS + b];
    mass_shape<double, DIM, false>(v);
    const double f = sig_s[j] * g.vol;
#pragma unroll
    for (int b = 0; b < NS; ++b) out[t * NS + b] = (T)(f * v[b]);
  }
}

// ---------------------------------------------------------------- sources
__global__ void k_rhs_volume(double *__restrict__ b, const double *__restrict__ q, const double *__restrict__ ipsi,
                             int A, Grid g) {
  const long long total = (long long)A * g.S;
  const double bint = g.vol / g.ns;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long a = t / g.S;
    const long long j = (t - a * g.S) / g.ns;
    b[t] = q ? q[j] * bint * ipsi[a] : 0.0;
  }
}

__global__ void k_rhs_face(double *__restrict__ b, const double *__restrict__ coef, const int *__restrict__ cells,
                           int ncells, const double *__restrict__ face_int, int A, Grid g) {
  const long long total = (long long)A * ncells;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long a = t / ncells;
    const int jc = cells[t - a * ncells];
    const double cf = coef[a];
    if (cf == 0.0) continue;
    for (int i = 0; i < g.ns; ++i) b[a * g.S + (long long)jc * g.ns + i] += cf * face_int[i];
  }
}

__global__ void k_detector(double *__restrict__ w, const double *__restrict__ ipsi, int A, Grid g, int lo0, int lo1,
                           int lo2, int hi0, int hi1, int hi2) {
  const long long total = (long long)A * g.S;
  const double bint = g.vol / g.ns;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long a = t / g.S;
    const long long j = (t - a * g.S) / g.ns;
    const int ix = (int)(j % g.n[0]), iy = (int)((j / g.n[0]) % g.n[1]), iz = (int)(j / ((long long)g.n[0] * g.n[1]));
    bool in = ix >= lo0 && ix <= hi0 && iy >= lo1 && iy <= hi1;
    if (g.dim == 3) in = in && iz >= lo2 && iz <= hi2;
    w[t] = in ? ipsi[a] * bint : 0.0;
  }
}

// grad_t[j] = -sum_q lambda_jq^T (N (x) M_q) phi_jq with M_q = Psi W Psi
template <int DIM>
__global__ void k_grad_t(const double *__restrict__ lam, const double *__restrict__ phi,
                         const double *__restrict__ w, int P, Grid g, double *__restrict__ gt) {
  constexpr int NS = 1 << DIM;
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < g.C;
       j += (long long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int q = 0; q < P; ++q) {
      double lv[3][NS], pv[3][NS];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        load_node_vec<double, NS>(lam + (3LL * q + m) * g.S + j * NS, lv[m]);
        load_node_vec<double, NS>(phi + (3LL * q + m) * g.S + j * NS, pv[m]);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double lk[NS], pk[NS];
#pragma unroll
        for (int b = 0; b < NS; ++b) {
          lk[b] = (lv[0][b] + lv[1][b] + lv[2][b] + 3.0 * lv[k][b]) * (1.0 / 6.0);
          pk[b] = (pv[0][b] + pv[1][b] + pv[2][b] + 3.0 * pv[k][b]) * (1.0 / 6.0);
        }
        mass_shape<double, DIM, false>(pk);
        double dd = 0.0;
#pragma unroll
        for (int b = 0; b < NS; ++b) dd += lk[b] * pk[b];
        acc += w[3 * q + k] * dd;
      }
    }
    gt[j] = -acc * g.vol;
  }
}

// grad_s[j] = sum_a lambda_aj^T N t_aj with t = S~ phi
template <int DIM>
__global__ void k_grad_s(const double *__restrict__ lam, const double *__restrict__ tt, int A, Grid g,
                         double *__restrict__ gs) {
  constexpr int NS = 1 << DIM;
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < g.C;
       j += (long long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int a = 0; a < A; ++a) {
      double lv[NS], tv[NS];
      load_node_vec<double, NS>(lam + (long long)a * g.S + j * NS, lv);
      load_node_vec<double, NS>(tt + (long long)a * g.S + j * NS, tv);
      mass_shape<double, DIM, false>(tv);
#pragma unroll
      for (int b = 0; b < NS; ++b) acc += lv[b] * tv[b];
    }
    gs[j] = acc * g.vol;
  }
}

// ----------------------------------------------------------------- BLAS-1
// BLAS-1 on long FP64 vectors: 16-byte accesses (two elements per lane),
// a grid-stride loop over pairs with the odd tail done by one lane.
__device__ __forceinline__ double block_sum(double acc) {
  __shared__ double red[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
  return t;
}

// partial[block] = sum x.y over the block's share
__global__ __launch_bounds__(kBlock) void k_dot_partial(const double *__restrict__ x, const double *__restrict__ y,
                                                        long long n, double *__restrict__ partial) {
  const long long n2 = n / 2;
  const double2 *x2 = reinterpret_cast<const double2 *>(x);
  const double2 *y2 = reinterpret_cast<const double2 *>(y);
  double a0 = 0.0, a1 = 0.0;
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n2; i += (long long)gridDim.x * kBlock) {
    const double2 u = x2[i], v = y2[i];
    a0 += u.x * v.x;
    a1 += u.y * v.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) a0 += x[n - 1] * y[n - 1];
  const double t = block_sum(a0 + a1);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_dot_final(const double *__restrict__ partial, int nb,
                                                      double *__restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) acc += partial[i];
  const double t = block_sum(acc);
  if (threadIdx.x == 0) *out = t;
}

__global__ void k_axpy(long long n, double a, const double *__restrict__ x, double *__restrict__ y) {
  const long long n2 = n / 2;
  const double2 *x2 = reinterpret_cast<const double2 *>(x);
  double2 *y2 = reinterpret_cast<double2 *>(y);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2; i += (long long)gridDim.x * blockDim.x) {
    const double2 u = x2[i];
    double2 v = y2[i];
    v.x += a * u.x;
    v.y += a * u.y;
    y2[i] = v;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) y[n - 1] += a * x[n - 1];
}

// y += sum_i c_i x_i for up to kMaxMulti vectors in one pass
struct MultiAxpyArgs {
  const double *x[kMaxMulti];
  double c[kMaxMulti];
  int k;
};

__global__ void k_multi_axpy(long long n, MultiAxpyArgs a, double *__restrict__ y) {
  const long long n2 = n / 2;
  double2 *y2 = reinterpret_cast<double2 *>(y);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2; i += (long long)gridDim.x * blockDim.x) {
    double2 v = y2[i];
    for (int q = 0; q < a.k; ++q) {
      const double2 u = reinterpret_cast<const double2 *>(a.x[q])[i];
      v.x += a.c[q] * u.x;
      v.y += a.c[q] * u.y;
    }
    y2[i] = v;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0)
    for (int q = 0; q < a.k; ++q) y[n - 1] += a.c[q] * a.x[q][n - 1];
}

// y += sum_i c_i x_i with FP32 vectors x_i (the flexible GMRES update from
// the FP32 preconditioned vectors), accumulated in FP64
struct MultiAxpyArgsF {
  const float *x[kMaxMulti];
  double c[kMaxMulti];
  int k;
};

__global__ void k_multi_axpy_f32(long long n, MultiAxpyArgsF a, double *__restrict__ y) {
  const long long n2 = n / 2;
  double2 *y2 = reinterpret_cast<double2 *>(y);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2; i += (long long)gridDim.x * blockDim.x) {
    double2 v = y2[i];
    for (int q = 0; q < a.k; ++q) {
      const float2 u = reinterpret_cast<const float2 *>(a.x[q])[i];
      v.x += a.c[q] * (double)u.x;
      v.y += a.c[q] * (double)u.y;
    }
    y2[i] = v;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0)
    for (int q = 0; q < a.k; ++q) y[n - 1] += a.c[q] * (double)a.x[q][n - 1];
}

// Several inner products in one pass (the projections of one Arnoldi step
// computed together, see the GMRES driver):
//   partial[q][block]     = x_q . y   (q < k)
//   partial[k + q][block] = x_q . z   (q < kz; with zlast, z is x_{k-1} and
//                                      is not read a second time)
struct MultiDotArgs {
  const double *x[kMaxMulti];
  const double *y, *z;
  int k, kz;
  bool zlast;
};

__global__ __launch_bounds__(kBlock) void k_multi_dot(long long n, MultiDotArgs a, double *__restrict__ partial) {
  const long long n2 = n / 2;
  double sy[kMaxMulti], sz[kMaxMulti];
#pragma unroll
  for (int q = 0; q < kMaxMulti; ++q) sy[q] = sz[q] = 0.0;
  const double2 *y2 = reinterpret_cast<const double2 *>(a.y);
  const double2 *z2 = reinterpret_cast<const double2 *>(a.z);
  const bool zsep = a.kz > 0 && !a.zlast;
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n2; i += (long long)gridDim.x * kBlock) {
    const double2 yy = y2[i];
    double2 xv[kMaxMulti];
#pragma unroll
    for (int q = 0; q < kMaxMulti; ++q)
      if (q < a.k) xv[q] = reinterpret_cast<const double2 *>(a.x[q])[i];
    double2 zz = make_double2(0.0, 0.0);
    if (zsep) zz = z2[i];
#pragma unroll
    for (int q = 0; q < kMaxMulti; ++q)
      if (a.zlast && q == a.k - 1) zz = xv[q];
#pragma unroll
    for (int q = 0; q < kMaxMulti; ++q)
      if (q < a.k) {
        sy[q] += xv[q].x * yy.x + xv[q].y * yy.y;
        if (q < a.kz) sz[q] += xv[q].x * zz.x + xv[q].y * zz.y;
      }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double yl = a.y[n - 1];
    const double zl = a.kz > 0 ? (a.zlast ? a.x[a.k - 1][n - 1] : a.z[n - 1]) : 0.0;
#pragma unroll
    for (int q = 0; q < kMaxMulti; ++q)
      if (q < a.k) {
        const double xl = a.x[q][n - 1];
        sy[q] += xl * yl;
        if (q < a.kz) sz[q] += xl * zl;
      }
  }
  double v[2 * kMaxMulti];
#pragma unroll
  for (int q = 0; q < kMaxMulti; ++q) {
    v[q] = sy[q];
    v[kMaxMulti + q] = sz[q];
  }
  // rows 0..k-1 then k..k+kz-1 of the partial table
  __shared__ double red[kBlock / 64][2 * kMaxMulti];
#pragma unroll
  for (int q = 0; q < 2 * kMaxMulti; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 2 * kMaxMulti; ++q) red[threadIdx.x >> 6][q] = v[q];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < a.k + a.kz) {
    const int col = t < a.k ? t : kMaxMulti + (t - a.k);
    double r = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) r += red[w][col];
    partial[(long long)t * gridDim.x + blockIdx.x] = r;
  }
}

// out[r] = sum of row r of a [rows][nb] partial table (one block per row)
__global__ __launch_bounds__(kBlock) void k_rows_final(const double *__restrict__ partial, int nb,
                                                       double *__restrict__ out) {
  const double *row = partial + (long long)blockIdx.x * nb;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) acc += row[i];
  const double t = block_sum(acc);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// y += sum_i c_i x_i (up to kMaxMulti vectors), and partial[block] = the
// block's share of |y|^2 after the update
__global__ __launch_bounds__(kBlock) void k_multi_axpy_norm(long long n, MultiAxpyArgs a, double *__restrict__ y,
                                                            double *__restrict__ partial) {
  const long long n2 = n / 2;
  double2 *y2 = reinterpret_cast<double2 *>(y);
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n2; i += (long long)gridDim.x * kBlock) {
    double2 v = y2[i];
    double2 xv[kMaxMulti];
#pragma unroll
    for (int q = 0; q < kMaxMulti; ++q)
      if (q < a.k) xv[q] = reinterpret_cast<const double2 *>(a.x[q])[i];
#pragma unroll
    for (int q = 0; q < kMaxMulti; ++q)
      if (q < a.k) {
        v.x += a.c[q] * xv[q].x;
        v.y += a.c[q] * xv[q].y;
      }
    y2[i] = v;
    acc += v.x * v.x + v.y * v.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double t = y[n - 1];
    for (int q = 0; q < a.k; ++q) t += a.c[q] * a.x[q][n - 1];
    y[n - 1] = t;
    acc += t * t;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void k_scal(long long n, double a, double *__restrict__ x) {
  const long long n2 = n / 2;
  double2 *x2 = reinterpret_cast<double2 *>(x);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2; i += (long long)gridDim.x * blockDim.x) {
    double2 v = x2[i];
    v.x *= a;
    v.y *= a;
    x2[i] = v;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) x[n - 1] *= a;
}

__global__ void k_axpby(long long n, double a, const double *__restrict__ x, double b, const double *__restrict__ y,
                        double *__restrict__ z) {
  const long long n2 = n / 2;
  const double2 *x2 = reinterpret_cast<const double2 *>(x);
  const double2 *y2 = reinterpret_cast<const double2 *>(y);
  double2 *z2 = reinterpret_cast<double2 *>(z);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2; i += (long long)gridDim.x * blockDim.x) {
    const double2 u = x2[i], v = y2[i];
    z2[i] = double2{a * u.x + b * v.x, a * u.y + b * v.y};
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) z[n - 1] = a * x[n - 1] + b * y[n - 1];
}

__global__ void k_fill_u32(unsigned *x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = 0u;
}

template <typename T>
__global__ void k_fill(T *x, long long n, T v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

int grid_for(long long n, int block = kBlock) {
  long long g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

// ------------------------------------------------------------- launchers
// LDS sweep: the compute lanes hold CPT cells of a plane each (cells
// tid + r tc), the compute waves cover the largest plane, the remaining
// waves of the NT-thread workgroup store; at least one store wave and at
// most 160 KB of LDS (staging, one or two plane buffers, plane offsets).
// Configurations in order of preference: one cell per lane in 1024
// threads; for 3-D FP32 planes beyond 960 cells two cells per lane (forward
// sweeps without s; registers allow no more in 1024 threads), or four per
// lane in 512 threads.  FP64 keeps one cell per lane: the register budget of
// more, with the single plane buffer such planes leave room for, spills.
struct LdsCfg {
  int cpt = 0, nt = 0, tc = 0;
  bool dbuf = false;
  size_t lds = 0;
};

static bool lds_config(int tsize, int dim, const Planes &pl, bool has_s, LdsCfg &cfg) {
  const int ns = 1 << dim;
  const int cands[3][2] = {{1, 1024}, {2, 1024}, {4, 512}};
  for (auto &cd : cands) {
    const int cpt = cd[0], nt = cd[1];
    if (cpt > 1 && (dim != 3 || tsize == 8)) continue;
    if (cpt == 2 && has_s) continue;
    const int tc = ((pl.max_plane + cpt - 1) / cpt + 63) / 64 * 64;
    if (tc > nt - 64) continue;
    const size_t stage = (size_t)(tc / 64) * (has_s ? 2 : 1) * 64 * tsize * ns;
    const size_t plane = ((size_t)tsize * ns + sizeof(int)) * (size_t)pl.max_plane;
    const size_t tail = sizeof(int) * (pl.nplanes + 1);
    if (stage + plane + tail > 160 * 1024) continue;
    cfg.cpt = cpt;
    cfg.nt = nt;
    cfg.tc = tc;
    // two plane buffers (one barrier per plane) where they fit, else one
    cfg.dbuf = stage + 2 * plane + tail <= 160 * 1024;
    cfg.lds = stage + (cfg.dbuf ? 2 : 1) * plane + tail;
    return true;
  }
  return false;
}

template <typename T, int DIM, bool ADJ, bool HAS_S, int CPT, int NT>
static void launch_sweep_lds_cfg(const SweepArgs<T> &a, int n_ord, const LdsCfg &cfg, bool pin, hipStream_t st) {
  auto fn = cfg.dbuf ? (pin ? k_sweep_lds<T, DIM, ADJ, HAS_S, true, !ADJ && !HAS_S, CPT, NT>
                            : k_sweep_lds<T, DIM, ADJ, HAS_S, true, false, CPT, NT>)
                     : (pin ? k_sweep_lds<T, DIM, ADJ, HAS_S, false, !ADJ && !HAS_S, CPT, NT>
                            : k_sweep_lds<T, DIM, ADJ, HAS_S, false, false, CPT, NT>);
  if (cfg.lds > 64 * 1024 &&
      hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg.lds) != hipSuccess)
    throw std::runtime_error("LDS sweep: cannot reserve its shared memory");
  hipLaunchKernelGGL(fn, dim3(n_ord), dim3(NT), cfg.lds, st, a, cfg.tc);
}

template <typename T, int DIM, bool ADJ, bool HAS_S>
static bool launch_sweep_lds(const SweepArgs<T> &a, int n_ord, hipStream_t st) {
  LdsCfg cfg;
  if (!a.sig_pl || !lds_config((int)sizeof(T), DIM, a.pl, HAS_S, cfg)) return false;
  // whole-cell accesses are 16-byte vector loads and stores
  auto aligned = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
  if (!aligned(a.f) || !aligned(a.u) || (a.s && !aligned(a.s))) return false;
  // right-hand side in plane layout: forward sweeps without s only
  const bool pin = a.plane_in && !ADJ && !HAS_S;
  if (a.plane_in && !pin) throw std::runtime_error("plane-layout input needs a forward sweep without s");
  if (cfg.cpt == 1) {
    launch_sweep_lds_cfg<T, DIM, ADJ, HAS_S, 1, 1024>(a, n_ord, cfg, pin, st);
    return true;
  }
  if constexpr (DIM == 3 && sizeof(T) == 4) {
    if (cfg.cpt == 2) {
      if constexpr (!HAS_S) {
        launch_sweep_lds_cfg<T, DIM, ADJ, HAS_S, 2, 1024>(a, n_ord, cfg, pin, st);
        return true;
      }
    } else {
      launch_sweep_lds_cfg<T, DIM, ADJ, HAS_S, 4, 512>(a, n_ord, cfg, pin, st);
      return true;
    }
  }
  throw std::runtime_error("internal: LDS sweep configuration without a kernel");
}

template <typename T>
bool sweep_lds_fits(const Planes &pl, const Grid &g, bool has_s) {
  LdsCfg cfg;
  return lds_config((int)sizeof(T), g.dim, pl, has_s, cfg);
}
template bool sweep_lds_fits<double>(const Planes &, const Grid &, bool);
template bool sweep_lds_fits<float>(const Planes &, const Grid &, bool);

struct PairCfg {
  int cpt = 0, nt = 0, tc = 0;
  bool dbuf = false;
  size_t lds = 0;
};

// Launch shape of the pair sweep: bricks per compute lane and threads (at
// least one store wave), one or two plane buffers in the 160 KB of LDS.
// Chosen by measurement (48^3 FP32: 2 bricks per lane and 768 threads,
// 3.2 ms; 1024 threads 5.7 ms (register cap), 4 per lane 13 ms, store
// waves' work done by the compute lanes themselves 3.4 ms).  FP64 bricks
// (128 bytes) take one per lane, 768 threads (512: 0.63 ms at 32^3
// against 0.52 ms).
static bool pair_config(int tsize, const Planes &bpl, PairCfg &cfg) {
  if (bpl.nplanes <= 0) return false;
  const int cands[4][2] = {{1, 512}, {1, 768}, {2, 768}, {1, 1024}};
  for (auto &cd : cands) {
    const int cpt = cd[0], nt = cd[1];
    if (tsize == 8 && !(cpt == 1 && nt == 768)) continue;
    const int tc = ((bpl.max_plane + cpt - 1) / cpt + 63) / 64 * 64;
    if (tc > nt - 64) continue;
    const size_t plane = ((size_t)tsize * 16 + sizeof(int)) * (size_t)bpl.max_plane;
    const size_t tail = sizeof(int) * (bpl.nplanes + 1);
    if (plane + tail > 160 * 1024) continue;
    cfg.cpt = cpt;
    cfg.nt = nt;
    cfg.tc = tc;
    cfg.dbuf = 2 * plane + tail <= 160 * 1024;
    cfg.lds = (cfg.dbuf ? 2 : 1) * plane + tail;
    return true;
  }
  return false;
}

template <typename T, bool HAS_S, int CPT, int NT, int MINW>
static void launch_pair_cfg(const SweepArgs<T> &a, int n_ord, const PairCfg &cfg, bool pin, hipStream_t st) {
  auto fn = cfg.dbuf ? (pin ? k_sweep_pair<T, HAS_S, true, !HAS_S, CPT, NT, MINW>
                            : k_sweep_pair<T, HAS_S, true, false, CPT, NT, MINW>)
                     : (pin ? k_sweep_pair<T, HAS_S, false, !HAS_S, CPT, NT, MINW>
                            : k_sweep_pair<T, HAS_S, false, false, CPT, NT, MINW>);
  if (cfg.lds > 64 * 1024 &&
      hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg.lds) != hipSuccess)
    throw std::runtime_error("pair sweep: cannot reserve its shared memory");
  hipLaunchKernelGGL(fn, dim3(n_ord), dim3(NT), cfg.lds, st, a, cfg.tc);
}

template <typename T, bool HAS_S>
static bool launch_sweep_pair(const SweepArgs<T> &a, int n_ord, hipStream_t st) {
  PairCfg cfg;
  if (!a.sig_pb || !pair_config((int)sizeof(T), a.bpl, cfg)) return false;
  auto aligned = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
  if (!aligned(a.f) || !aligned(a.u) || (a.s && !aligned(a.s))) return false;
  if (a.plane_in && HAS_S) throw std::runtime_error("plane-layout input needs a forward sweep without s");
  const bool pin = a.plane_in;
  if (cfg.cpt == 1 && cfg.nt == 512) {
    // FP32: two workgroups per CU (registers for four waves per SIMD)
    if constexpr (sizeof(T) == 4)
      launch_pair_cfg<T, HAS_S, 1, 512, 4>(a, n_ord, cfg, pin, st);
    else
      throw std::runtime_error("internal: FP64 pair sweep with 512 threads");
  } else if (cfg.cpt == 1 && cfg.nt == 768) {
    launch_pair_cfg<T, HAS_S, 1, 768, 3>(a, n_ord, cfg, pin, st);
  } else if (cfg.cpt == 1 && cfg.nt == 1024) {
    if constexpr (sizeof(T) == 4)
      launch_pair_cfg<T, HAS_S, 1, 1024, 4>(a, n_ord, cfg, pin, st);
    else
      throw std::runtime_error("internal: FP64 pair sweep with 1024 threads");
  } else if (cfg.cpt == 2 && cfg.nt == 768) {
    if constexpr (sizeof(T) == 4)
      launch_pair_cfg<T, HAS_S, 2, 768, 3>(a, n_ord, cfg, pin, st);
    else
      throw std::runtime_error("internal: FP64 pair sweep with two bricks per lane");
  } else {
    throw std::runtime_error("internal: pair sweep configuration without a kernel");
  }
  return true;
}

template <typename T>
bool sweep_pair_fits(const Planes &bpl) {
  PairCfg cfg;
  return pair_config((int)sizeof(T), bpl, cfg);
}
template bool sweep_pair_fits<double>(const Planes &);
template bool sweep_pair_fits<float>(const Planes &);

template <typename T, int DIM, bool ADJ>
static void launch_sweep_r(const SweepArgs<T> &a, int n_ord, hipStream_t st) {
  if constexpr (DIM == 3 && !ADJ) {
    // forward sweeps of prepared right-hand sides (no separate scatter term)
    if (a.bpl.nplanes > 0 && !a.s) {
      if (launch_sweep_pair<T, false>(a, n_ord, st)) return;
      // with pairs the plane layout is the brick slot order: no other kernel reads it
      if (a.plane_in) throw std::runtime_error("plane-layout input needs the pair sweep");
    }
  }
  if (a.s ? launch_sweep_lds<T, DIM, ADJ, true>(a, n_ord, st) : launch_sweep_lds<T, DIM, ADJ, false>(a, n_ord, st))
    return;
  if (a.plane_in) throw std::runtime_error("plane-layout input needs the LDS sweep");
  const int R = (a.pl.max_plane + kSweepThreads - 1) / kSweepThreads;
  // register prefetch of the next plane when a thread owns one cell per
  // plane; with more cells per thread the prefetch buffers would halve the
  // workgroups resident per CU, so those variants load at use
  if (R <= 1)
    hipLaunchKernelGGL((k_sweep<T, DIM, ADJ, 1, true>), dim3(n_ord), dim3(kSweepThreads), 0, st, a);
  else if (R <= 2)
    hipLaunchKernelGGL((k_sweep<T, DIM, ADJ, 2, false>), dim3(n_ord), dim3(kSweepThreads), 0, st, a);
  else if (R <= 4)
    hipLaunchKernelGGL((k_sweep<T, DIM, ADJ, 4, false>), dim3(n_ord), dim3(kSweepThreads), 0, st, a);
  else if (R <= 8)
    hipLaunchKernelGGL((k_sweep<T, DIM, ADJ, 8, false>), dim3(n_ord), dim3(kSweepThreads), 0, st, a);
  else
    throw std::runtime_error("sweep plane larger than 4096 cells");
}

template <typename T>
void launch_sweep(const SweepArgs<T> &a, int n_ord, bool adjoint, hipStream_t st) {
  if (a.g.dim == 3) {
    if (adjoint)
      launch_sweep_r<T, 3, true>(a, n_ord, st);
    else
      launch_sweep_r<T, 3, false>(a, n_ord, st);
  } else {
    if (adjoint)
      launch_sweep_r<T, 2, true>(a, n_ord, st);
    else
      launch_sweep_r<T, 2, false>(a, n_ord, st);
  }
}
template void launch_sweep<double>(const SweepArgs<double> &, int, bool, hipStream_t);

void launch_sigma_planes(const double *sig_t, const double *sig_s, const Planes &pl, const Grid &g, double *out,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_sigma_planes, dim3(grid_for(8 * g.C)), dim3(kBlock), 0, st, sig_t, sig_s, pl, g, out);
}
template void launch_sweep<float>(const SweepArgs<float> &, int, bool, hipStream_t);

// Threads per workgroup of the coarse Gauss-Seidel launch (cells per
// workgroup and round = threads / 2^dim).
static int g_gs_block_threads = 256;
static int gs_block_threads() { return g_gs_block_threads; }

void launch_coarse_flow(const double *f, double *u, const double *G, const double *sig_t, const double *sig_s,
                        const OrdInfo *ord, const Planes &pl, const Grid &g, const int *wave_off, const int *slots,
                        int waves, bool adjoint, unsigned *cnt, int *err, hipStream_t st) {
  launch_fill<double>(u, 24LL * g.S, 0.0, st);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(g.C)), dim3(kBlock), 0, st, cnt, g.C);
  void *fn = g.dim == 3 ? (adjoint ? (void *)k_gs_flow<3, true> : (void *)k_gs_flow<3, false>)
                        : (adjoint ? (void *)k_gs_flow<2, true> : (void *)k_gs_flow<2, false>);
  const int blocks = (waves + 3) / 4;
  void *args[] = {(void *)&f,     (void *)&u,     (void *)&G,   (void *)&sig_t, (void *)&sig_s,
                  (void *)&ord,   (void *)&pl,    (void *)&g,   (void *)&wave_off, (void *)&slots,
                  (void *)&waves, (void *)&cnt,   (void *)&err};
  if (hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(256), args, 0, st) != hipSuccess)
    throw std::runtime_error("cooperative launch of the Gauss-Seidel solve failed");
}

void launch_coarse_brick(const double *f, double *u, const double *G, const double *sig_t, const double *sig_s,
                         const OrdInfo *ord, const Grid &g, const int *wave_off, const int *slots, int waves,
                         bool adjoint, unsigned *cnt, long long nbricks, int *err, hipStream_t st) {
  if (g.dim != 3 || (g.n[0] | g.n[1] | g.n[2]) & 1) throw std::runtime_error("brick Gauss-Seidel needs even 3-D grids");
  launch_fill<double>(u, 24LL * g.S, 0.0, st);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nbricks)), dim3(kBlock), 0, st, cnt, nbricks);
  void *args[] = {(void *)&f,   (void *)&u,        (void *)&G,     (void *)&sig_t, (void *)&sig_s,
                  (void *)&ord, (void *)&g,        (void *)&wave_off, (void *)&slots, (void *)&waves,
                  (void *)&cnt, (void *)&err};
  // one workgroup of three waves per slot list
  void *fn = adjoint ? (void *)k_gs_brick<true> : (void *)k_gs_brick<false>;
  if (hipLaunchCooperativeKernel(fn, dim3(waves), dim3(192), args, 0, st) != hipSuccess)
    throw std::runtime_error("cooperative launch of the Gauss-Seidel solve failed");
}

int coarse_brick_capacity() {
  // workgroups of both brick kernels that stay co-resident on the device
  // (0 without a device)
  int dev = 0, ncu = 0, a = 0, b = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, (const void *)k_gs_brick<false>, 192, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void *)k_gs_brick<true>, 192, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return ncu * std::min(a, b);
}

void launch_coarse_gs(const double *f, double *u, const double *G, const double *sig_t, const double *sig_s,
                      const OrdInfo *ord, const Planes &pl, const Grid &g, const int *step_off, const int *items,
                      int nsteps, int max_items, bool adjoint, unsigned *bar_arrive, unsigned *bar_release,
                      int *bar_err, int max_blocks, unsigned gen0, bool coh, hipStream_t st) {
  launch_fill<double>(u, 24LL * g.S, 0.0, st);
  const int tb = gs_block_threads();
  void *fn = nullptr;
#define TR_GS_FN(TB, COH)                                                                          \
  (g.dim == 3 ? (adjoint ? (void *)k_gs_solve<3, true, TB, COH> : (void *)k_gs_solve<3, false, TB, COH>) \
              : (adjoint ? (void *)k_gs_solve<2, true, TB, COH> : (void *)k_gs_solve<2, false, TB, COH>))
  if (coh)
    fn = tb == 1024 ? TR_GS_FN(1024, true) : tb == 512 ? TR_GS_FN(512, true) : TR_GS_FN(256, true);
  else
    fn = tb == 1024 ? TR_GS_FN(1024, false) : tb == 512 ? TR_GS_FN(512, false) : TR_GS_FN(256, false);
#undef TR_GS_FN
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, tb, 0) != hipSuccess || per_cu < 1)
    throw std::runtime_error("cannot size the cooperative Gauss-Seidel launch");
  const int cpb = tb / g.ns;
  int blocks = (max_items + cpb - 1) / cpb;
  blocks = std::max(1, std::min(std::min(blocks, ncu * per_cu), max_blocks));
  GridBarrier gb{bar_arrive, bar_release, bar_err};
  void *args[] = {(void *)&f,    (void *)&u,     (void *)&G,        (void *)&sig_t, (void *)&sig_s,
                  (void *)&ord,  (void *)&pl,    (void *)&g,        (void *)&step_off, (void *)&items,
                  (void *)&nsteps, (void *)&gb, (void *)&gen0};
  if (hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(tb), args, 0, st) != hipSuccess)
    throw std::runtime_error("cooperative launch of the Gauss-Seidel solve failed");
}

template <typename Tin, typename Tout>
void launch_convert(const Tin *in, Tout *out, int P, long long S, const double *pre, const double *post,
                    hipStream_t st, double scale, double *out64) {
  const long long n = (long long)P * S;
  if (n >= (1LL << 32) - kBlock) throw std::runtime_error("conversion: patches x spatial dofs must be below 2^32");
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, in, out,
                     P, S, pre, post, scale, out64);
}
template <typename Tin, typename Tout>
void launch_convert_minv(const Tin *in, Tout *out, int P, const Grid &g, const double *pre, const double *post,
                         hipStream_t st, const int *pos, const OrdInfo *ord, double scale) {
  const long long n = (long long)P * g.S;
  if (n >= (1LL << 32) - kBlock) throw std::runtime_error("conversion: patches x spatial dofs must be below 2^32");
  const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
  if (g.dim == 3)
    hipLaunchKernelGGL((k_convert_minv<Tin, Tout, 3>), grid, dim3(kBlock), 0, st, in, out, P, g, pre, post, pos, ord,
                       scale);
  else
    hipLaunchKernelGGL((k_convert_minv<Tin, Tout, 2>), grid, dim3(kBlock), 0, st, in, out, P, g, pre, post, pos, ord,
                       scale);
}
template void launch_convert_minv<double, double>(const double *, double *, int, const Grid &, const double *,
                                                  const double *, hipStream_t, const int *, const OrdInfo *, double);
template void launch_convert_minv<double, float>(const double *, float *, int, const Grid &, const double *,
                                                 const double *, hipStream_t, const int *, const OrdInfo *, double);
template void launch_convert_minv<float, float>(const float *, float *, int, const Grid &, const double *,
                                                const double *, hipStream_t, const int *, const OrdInfo *, double);
template void launch_convert<double, double>(const double *, double *, int, long long, const double *,
                                             const double *, hipStream_t, double, double *);
template void launch_convert<double, float>(const double *, float *, int, long long, const double *, const double *,
                                            hipStream_t, double, double *);
template void launch_convert<float, double>(const float *, double *, int, long long, const double *, const double *,
                                            hipStream_t, double, double *);
template void launch_convert<float, float>(const float *, float *, int, long long, const double *, const double *,
                                           hipStream_t, double, double *);

template <typename Tin, typename Tout>
void launch_restrict(const Tin *s_new, const Tin *s_prev, Tout *fc, const double *R, const int *first_child,
                     const int *n_child, int Pc, const double *sig_s, bool apply_sn, const Grid &g,
                     hipStream_t st, const int *pos, const OrdInfo *cord) {
  // one lane per (coarse patch, spatial dof), 32-bit indices
  const long long n = (long long)Pc * g.S;
  if (n >= (1LL << 32) - kBlock) throw std::runtime_error("restriction: coarse patches x spatial dofs must be below 2^32");
  const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
  if (g.dim == 3)
    hipLaunchKernelGGL((k_restrict<Tin, Tout, 3>), grid, dim3(kBlock), 0, st, s_new, s_prev, fc, R, first_child,
                       n_child, Pc, sig_s, (int)apply_sn, g, pos, cord);
  else
    hipLaunchKernelGGL((k_restrict<Tin, Tout, 2>), grid, dim3(kBlock), 0, st, s_new, s_prev, fc, R, first_child,
                       n_child, Pc, sig_s, (int)apply_sn, g, pos, cord);
}
#define TR_INST_RESTRICT(TI, TO)                                                                               \
  template void launch_restrict<TI, TO>(const TI *, const TI *, TO *, const double *, const int *, const int *, \
                                        int, const double *, bool, const Grid &, hipStream_t, const int *,     \
                                        const OrdInfo *);
TR_INST_RESTRICT(double, double)
TR_INST_RESTRICT(float, float)
TR_INST_RESTRICT(float, double)
TR_INST_RESTRICT(double, float)

template <typename Tin, typename Tout>
void launch_prolong(const Tin *uc, Tout *uf, const double *Pblk, const int *first_child, const int *n_child, int Pc,
                    long long S, bool add, hipStream_t st) {
  const long long n = (long long)Pc * S;
  if (n >= (1LL << 32) - kBlock) throw std::runtime_error("prolongation: coarse patches x spatial dofs must be below 2^32");
  hipLaunchKernelGGL((k_prolong<Tin, Tout>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, uc, uf,
                     Pblk, first_child, n_child, Pc, S, (int)add);
}
#define TR_INST_PROLONG(TI, TO)                                                                                    \
  template void launch_prolong<TI, TO>(const TI *, TO *, const double *, const int *, const int *, int, long long, \
                                       bool, hipStream_t);
TR_INST_PROLONG(double, double)
TR_INST_PROLONG(float, float)
TR_INST_PROLONG(double, float)
TR_INST_PROLONG(float, double)

template <typename TX>
static void launch_apply_t(const TX *x, const double *s, double *y, const double *sig_t, const double *sig_s,
                           const OrdInfo *ord, const double *w, int P, const Grid &g, bool adjoint, hipStream_t st) {
  // one (patch, cell) per thread; the grid a multiple of the 8 XCDs
  const long long cells = (long long)P * g.C;
  if (cells >= (1LL << 31)) throw std::runtime_error("operator apply: patches x cells must be below 2^31");
  const int per_xcd = (int)((cells + 8LL * kBlock - 1) / (8LL * kBlock));
  const dim3 grid(8 * per_xcd);
  if (g.dim == 3) {
    if (adjoint)
      hipLaunchKernelGGL((k_apply_cells<3, true, TX>), grid, dim3(kBlock), 0, st, x, s, y, sig_t, sig_s, ord, w, P, g,
                         per_xcd);
    else
      hipLaunchKernelGGL((k_apply_cells<3, false, TX>), grid, dim3(kBlock), 0, st, x, s, y, sig_t, sig_s, ord, w, P,
                         g, per_xcd);
  } else {
    if (adjoint)
      hipLaunchKernelGGL((k_apply_cells<2, true, TX>), grid, dim3(kBlock), 0, st, x, s, y, sig_t, sig_s, ord, w, P, g,
                         per_xcd);
    else
      hipLaunchKernelGGL((k_apply_cells<2, false, TX>), grid, dim3(kBlock), 0, st, x, s, y, sig_t, sig_s, ord, w, P,
                         g, per_xcd);
  }
}
void launch_apply(const double *x, const double *s, double *y, const double *sig_t, const double *sig_s,
                  const OrdInfo *ord, const double *w, int P, const Grid &g, bool adjoint, hipStream_t st) {
  launch_apply_t(x, s, y, sig_t, sig_s, ord, w, P, g, adjoint, st);
}
void launch_apply(const float *x, const double *s, double *y, const double *sig_t, const double *sig_s,
                  const OrdInfo *ord, const double *w, int P, const Grid &g, bool adjoint, hipStream_t st) {
  launch_apply_t(x, s, y, sig_t, sig_s, ord, w, P, g, adjoint, st);
}

template <typename T>
void launch_scale_sn(const T *in, T *out, const double *sig_s, int A, const Grid &g, hipStream_t st) {
  const int grid = grid_for((long long)A * g.C);
  if (g.dim == 3)
    hipLaunchKernelGGL((k_scale_sn<T, 3>), dim3(grid), dim3(kBlock), 0, st, in, out, sig_s, A, g);
  else
    hipLaunchKernelGGL((k_scale_sn<T, 2>), dim3(grid), dim3(kBlock), 0, st, in, out, sig_s, A, g);
}
template void launch_scale_sn<double>(const double *, double *, const double *, int, const Grid &, hipStream_t);
template void launch_scale_sn<float>(const float *, float *, const double *, int, const Grid &, hipStream_t);

void launch_rhs_volume(double *b, const double *q, const double *ipsi, int A, const Grid &g, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs_volume, dim3(grid_for((long long)A * g.S)), dim3(kBlock), 0, st, b, q, ipsi, A, g);
}

void launch_rhs_face(double *b, const double *coef, const int *cells, int ncells, const double *face_int, int A,
                     const Grid &g, hipStream_t st) {
  if (ncells <= 0) return;
  hipLaunchKernelGGL(k_rhs_face, dim3(grid_for((long long)A * ncells)), dim3(kBlock), 0, st, b, coef, cells, ncells,
                     face_int, A, g);
}

void launch_detector(double *w, const double *ipsi, int A, const Grid &g, const int lo[3], const int hi[3],
                     hipStream_t st) {
  hipLaunchKernelGGL(k_detector, dim3(grid_for((long long)A * g.S)), dim3(kBlock), 0, st, w, ipsi, A, g, lo[0],
                     lo[1], lo[2], hi[0], hi[1], hi[2]);
}

void launch_grad_t(const double *lam, const double *phi, const double *w, int P, const Grid &g, double *gt,
                   hipStream_t st) {
  const int grid = grid_for(g.C, 64);
  if (g.dim == 3)
    hipLaunchKernelGGL((k_grad_t<3>), dim3(grid), dim3(64), 0, st, lam, phi, w, P, g, gt);
  else
    hipLaunchKernelGGL((k_grad_t<2>), dim3(grid), dim3(64), 0, st, lam, phi, w, P, g, gt);
}

void launch_grad_s(const double *lam, const double *t, int A, const Grid &g, double *gs, hipStream_t st) {
  const int grid = grid_for(g.C, 64);
  if (g.dim == 3)
    hipLaunchKernelGGL((k_grad_s<3>), dim3(grid), dim3(64), 0, st, lam, t, A, g, gs);
  else
    hipLaunchKernelGGL((k_grad_s<2>), dim3(grid), dim3(64), 0, st, lam, t, A, g, gs);
}

void launch_dot_partial(const double *x, const double *y, long long n, double *partial, int nblocks,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial, dim3(nblocks), dim3(kBlock), 0, st, x, y, n, partial);
}
void launch_dot_final(const double *partial, int nblocks, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, st, partial, nblocks, out);
}
// BLAS-1 launches: 16-byte accesses need 16-byte aligned vectors (every
// vector the library passes here is a device allocation or a caller buffer
// checked at the entry point)
static int blas_grid(long long n) {
  long long g = (n / 2 + kBlock - 1) / kBlock;
  return (int)std::max(1LL, std::min(g, 8192LL));
}
void launch_axpy(long long n, double a, const double *x, double *y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(blas_grid(n)), dim3(kBlock), 0, st, n, a, x, y);
}
void launch_multi_axpy(long long n, int k, const double *const *x, const double *c, double *y, hipStream_t st) {
  for (int q0 = 0; q0 < k; q0 += kMaxMulti) {
    MultiAxpyArgs a{};
    a.k = std::min(kMaxMulti, k - q0);
    for (int q = 0; q < a.k; ++q) {
      a.x[q] = x[q0 + q];
      a.c[q] = c[q0 + q];
    }
    hipLaunchKernelGGL(k_multi_axpy, dim3(blas_grid(n)), dim3(kBlock), 0, st, n, a, y);
  }
}
void launch_multi_axpy_f32(long long n, int k, const float *const *x, const double *c, double *y, hipStream_t st) {
  for (int q0 = 0; q0 < k; q0 += kMaxMulti) {
    MultiAxpyArgsF a{};
    a.k = std::min(kMaxMulti, k - q0);
    for (int q = 0; q < a.k; ++q) {
      a.x[q] = x[q0 + q];
      a.c[q] = c[q0 + q];
    }
    hipLaunchKernelGGL(k_multi_axpy_f32, dim3(blas_grid(n)), dim3(kBlock), 0, st, n, a, y);
  }
}
// Workgroups of a multi-vector pass: one resident round (a second, partly
// filled round of long grid-stride workgroups costs more than it hides),
// at most nblocks (the partial buffer's capacity).
static int resident_blocks(const void *fn, int nblocks) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess || per_cu < 1)
    return nblocks;
  return std::max(1, std::min(nblocks, ncu * per_cu));
}

void launch_multi_dot(long long n, int k, const double *const *x, const double *y, int kz, const double *z,
                      double *partial, int nblocks, double *out, hipStream_t st) {
  static const int resident = resident_blocks((const void *)k_multi_dot, 1 << 30);
  nblocks = std::min(nblocks, resident);
  if (k < 1 || k > kMaxMulti || kz < 0 || kz > k) throw std::runtime_error("multi-dot: bad vector count");
  MultiDotArgs a{};
  a.k = k;
  a.kz = kz;
  for (int q = 0; q < k; ++q) a.x[q] = x[q];
  a.y = y;
  a.z = z;
  a.zlast = kz > 0 && z == x[k - 1];
  hipLaunchKernelGGL(k_multi_dot, dim3(nblocks), dim3(kBlock), 0, st, n, a, partial);
  hipLaunchKernelGGL(k_rows_final, dim3(k + kz), dim3(kBlock), 0, st, partial, nblocks, out);
}
void launch_multi_axpy_norm(long long n, int k, const double *const *x, const double *c, double *y,
                            double *partial, int nblocks, double *out, hipStream_t st) {
  static const int resident = resident_blocks((const void *)k_multi_axpy_norm, 1 << 30);
  nblocks = std::min(nblocks, resident);
  // all but the last group of vectors without the norm
  int q0 = 0;
  for (; k - q0 > kMaxMulti; q0 += kMaxMulti) launch_multi_axpy(n, kMaxMulti, x + q0, c + q0, y, st);
  MultiAxpyArgs a{};
  a.k = k - q0;
  for (int q = 0; q < a.k; ++q) {
    a.x[q] = x[q0 + q];
    a.c[q] = c[q0 + q];
  }
  hipLaunchKernelGGL(k_multi_axpy_norm, dim3(nblocks), dim3(kBlock), 0, st, n, a, y, partial);
  hipLaunchKernelGGL(k_rows_final, dim3(1), dim3(kBlock), 0, st, partial, nblocks, out);
}
void launch_scal(long long n, double a, double *x, hipStream_t st) {
  hipLaunchKernelGGL(k_scal, dim3(blas_grid(n)), dim3(kBlock), 0, st, n, a, x);
}
void launch_axpby(long long n, double a, const double *x, double b, const double *y, double *z, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(blas_grid(n)), dim3(kBlock), 0, st, n, a, x, b, y, z);
}
template <typename T>
void launch_fill(T *x, long long n, T v, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n)), dim3(kBlock), 0, st, x, n, v);
}
void launch_fill_u32(unsigned *x, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kBlock), 0, st, x, n);
}
template void launch_fill<double>(double *, long long, double, hipStream_t);
template void launch_fill<float>(float *, long long, float, hipStream_t);

}  // namespace tr
