// Internal declarations shared by the library's host code and kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tr {

// Per-ordinate data of an angular level.
struct alignas(16) OrdInfo {
  double c[3];   // |Omega_xi| / h_xi
  double a[3];   // |Omega_xi|
  int flip;      // bit xi set when Omega_xi < 0
  int patch;
};

struct Grid {
  int dim, ns;
  int n[3];
  double h[3];
  double vol;         // cell volume
  long long C, S;     // cells, spatial dofs
};

// Sweep schedule: cells of the (+,+,+) orientation grouped by diagonal
// plane; a cell is packed as ix | iy << 10 | iz << 20.
struct Planes {
  const int *cells;
  const int *off;     // [nplanes + 1]
  int nplanes;
  int max_plane;
  // Per cell-list entry: {packed cell, position of the neighbour along
  // x, y, z within the adjacent plane, or -1 at the boundary}; link[0] the
  // upwind neighbours (previous plane), link[1] the downwind ones (next plane).
  const int4 *link[2];
};

template <typename T>
struct SweepArgs {
  const T *f;           // [A][S] right-hand side in ordinate form
  const T *s;           // [A][S] scatter moments G u (may be null)
  T *u;                 // [A][S] ordinate values (output)
  const double *sig_t, *sig_s;
  // sigma_t and sigma_s per orientation in cell-list order:
  // [2][8][cells], index [which][flip][list index]
  const double *sig_pl;
  const OrdInfo *ord;
  Planes pl;
  Grid g;
  // f is stored in plane order: ordinate k's cell at list position i of its
  // orientation's sweep occupies f[k][i][node] (forward sweeps without s)
  bool plane_in = false;
  // Brick schedule of the pair sweep (3-D grids with an even number of
  // cells along x; nplanes = 0 otherwise): bricks of the two cells 2b, 2b+1
  // of the (+,+,+) frame, packed b | iy << 10 | iz << 20, grouped by
  // diagonal plane b + iy + iz; link[0] per brick = {packed brick, position
  // of its x, y, z upwind bricks in the previous plane or -1}.  With pairs
  // the plane layout holds brick i's cells at positions 2i, 2i + 1 (slot
  // order of the sweep frame), and sig_pb the cross sections in that order.
  Planes bpl{};
  const double *sig_pb = nullptr;
};

// Sweep-input ("plane") layout: pos[flip][cell] = the cell's position in
// the sweep list of orientation flip ([8][C], device).  Writers of sweep
// inputs store ordinate k's cell j at position pos[ord[k].flip][j].

// Whether the LDS sweep (the only one that reads the plane layout) runs
// for this level and element type.
template <typename T>
bool sweep_lds_fits(const Planes &pl, const Grid &g, bool has_s);
// Whether the pair sweep runs forward sweeps of element type T on the
// brick schedule bpl.
template <typename T>
bool sweep_pair_fits(const Planes &bpl);

// Workgroups of the brick Gauss-Seidel kernels that stay co-resident on the
// current device (0 when no device answers).
int coarse_brick_capacity();

// Fill SweepArgs::sig_pl from the per-cell cross sections.
void launch_sigma_planes(const double *sig_t, const double *sig_s, const Planes &pl, const Grid &g, double *out,
                         hipStream_t st);

// ------------------------------------------------------------- launchers
template <typename T>
void launch_sweep(const SweepArgs<T> &a, int n_ord, bool adjoint, hipStream_t st);

// nu Gauss-Seidel sweeps on T_0 from zero, as one cooperative launch over a
// precomputed step schedule (items = (octant << 28) | cell-list index).
// The grid barrier uses bar_arrive[max_blocks], bar_release[1] and bar_err[1]
// (zeroed once); generations continue from gen0, which the caller advances
// by nsteps per launch.  bar_err != 0 after the launch means a barrier timed out.
// The same solve without grid barriers (per-cell update counters cnt[C],
// zeroed here; err as above): wave w runs slots wave_off[w] .. wave_off[w+1]
// of 64 / 2^dim items each (octant << 29 | count << 22 | list index, or -1).
void launch_coarse_flow(const double *f, double *u, const double *G, const double *sig_t, const double *sig_s,
                        const OrdInfo *ord, const Planes &pl, const Grid &g, const int *wave_off, const int *slots,
                        int waves, bool adjoint, unsigned *cnt, int *err, hipStream_t st);
// The same solve over 2 x 2 x 2 bricks (3-D, even grids): waves = slot
// lists, one workgroup of three waves each; cnt[nbricks] zeroed here.
void launch_coarse_brick(const double *f, double *u, const double *G, const double *sig_t, const double *sig_s,
                         const OrdInfo *ord, const Grid &g, const int *wave_off, const int *slots, int waves,
                         bool adjoint, unsigned *cnt, long long nbricks, int *err, hipStream_t st);
void launch_coarse_gs(const double *f, double *u, const double *G, const double *sig_t, const double *sig_s,
                      const OrdInfo *ord, const Planes &pl, const Grid &g, const int *step_off, const int *items,
                      int nsteps, int max_items, bool adjoint, unsigned *bar_arrive, unsigned *bar_release,
                      int *bar_err, int max_blocks, unsigned gen0, bool coh, hipStream_t st);

// out[a][s] = post[a] * sum_m Psi^{-1}[k(a)][m] * pre[3p+m] * scale * in[3p+m][s];
// out64 (optional): the same rounded values widened to FP64
template <typename Tin, typename Tout>
void launch_convert(const Tin *in, Tout *out, int P, long long S, const double *pre, const double *post,
                    hipStream_t st, double scale = 1.0, double *out64 = nullptr);
// The same conversion followed by the inverse cell mass matrix per ordinate:
// a forward right-hand side in prepared form f~ = N^{-1} f (the form every
// forward sweep, forward coarse solve and forward restriction works in).
template <typename Tin, typename Tout>
void launch_convert_minv(const Tin *in, Tout *out, int P, const Grid &g, const double *pre, const double *post,
                         hipStream_t st, const int *pos = nullptr, const OrdInfo *ord = nullptr, double scale = 1.0);

// Restriction to level l-1: fc[p] = sum_children R_c (sigma_s N (s_new - s_prev))_c
// (apply_sn = 0: plain fc[p] = sum_children R_c in_c).
template <typename Tin, typename Tout>
void launch_restrict(const Tin *s_new, const Tin *s_prev, Tout *fc, const double *R, const int *first_child,
                     const int *n_child, int Pc, const double *sig_s, bool apply_sn, const Grid &g,
                     hipStream_t st, const int *pos = nullptr, const OrdInfo *cord = nullptr);

// Prolongation: uf[c] (+)= P_c uc[p] for the children c of every coarse
// patch p (first_child[p] .. + n_child[p]), Pc coarse patches
template <typename Tin, typename Tout>
void launch_prolong(const Tin *uc, Tout *uf, const double *Pblk, const int *first_child, const int *n_child, int Pc,
                    long long S, bool add, hipStream_t st);

// y = L x - sigma_s N s  (canonical FP64, s = S~ x); adjoint: L^T x - sigma_s N s.
// The float form reads an FP32 x (its values widened exactly to FP64).
void launch_apply(const double *x, const double *s, double *y, const double *sig_t, const double *sig_s,
                  const OrdInfo *ord, const double *w, int P, const Grid &g, bool adjoint, hipStream_t st);
void launch_apply(const float *x, const double *s, double *y, const double *sig_t, const double *sig_s,
                  const OrdInfo *ord, const double *w, int P, const Grid &g, bool adjoint, hipStream_t st);

// out[a][j][i] = sigma_s[j] vol Nshape(in[a][j][.])[i]
template <typename T>
void launch_scale_sn(const T *in, T *out, const double *sig_s, int A, const Grid &g, hipStream_t st);

void launch_rhs_volume(double *b, const double *q, const double *ipsi, int A, const Grid &g, hipStream_t st);
void launch_rhs_face(double *b, const double *coef, const int *cells, int ncells, const double *face_int, int A,
                     const Grid &g, hipStream_t st);
void launch_detector(double *w, const double *ipsi, int A, const Grid &g, const int lo[3], const int hi[3],
                     hipStream_t st);
void launch_grad_t(const double *lam, const double *phi, const double *w, int P, const Grid &g, double *gt,
                   hipStream_t st);
void launch_grad_s(const double *lam, const double *t, int A, const Grid &g, double *gs, hipStream_t st);

// BLAS-1 (FP64) and helpers
void launch_dot_partial(const double *x, const double *y, long long n, double *partial, int nblocks,
                        hipStream_t st);
void launch_dot_final(const double *partial, int nblocks, double *out, hipStream_t st);
void launch_axpy(long long n, double a, const double *x, double *y, hipStream_t st);
void launch_scal(long long n, double a, double *x, hipStream_t st);
// y += sum_q c[q] x[q] (host arrays of k device vectors and coefficients)
void launch_multi_axpy(long long n, int k, const double *const *x, const double *c, double *y, hipStream_t st);
// the same with FP32 vectors x (FP64 accumulation)
void launch_multi_axpy_f32(long long n, int k, const float *const *x, const double *c, double *y, hipStream_t st);
// inner products x_q . y (q < k) and x_q . z (q < kz), k <= 16, into
// out[0..k) and out[k..k+kz); partial holds (k + kz) x nblocks doubles
void launch_multi_dot(long long n, int k, const double *const *x, const double *y, int kz, const double *z,
                      double *partial, int nblocks, double *out, hipStream_t st);
// y += sum_q c_q x_q (any k >= 1), then out[0] = |y|^2; partial holds nblocks doubles
void launch_multi_axpy_norm(long long n, int k, const double *const *x, const double *c, double *y,
                            double *partial, int nblocks, double *out, hipStream_t st);
void launch_axpby(long long n, double a, const double *x, double b, const double *y, double *z, hipStream_t st);
template <typename T>
void launch_fill(T *x, long long n, T v, hipStream_t st);
void launch_fill_u32(unsigned *x, long long n, hipStream_t st);  // x[0..n) = 0

// C[M][N] = A[M][K] * B[K][N]   (row-major; ld of B and C is N)
// C[M][N] = A[M][K] B[K][N] on the matrix cores; with bias / colscale:
// C = bias + colscale[c / cell] * (A B) per column c.
template <typename T>
void launch_gemm(const T *A, const T *B, T *C, int M, int N, int K, hipStream_t st, const T *bias = nullptr,
                 const double *colscale = nullptr, int cell = 8,
                 const int *pos = nullptr, const OrdInfo *rord = nullptr);
// Row map of the octant-group form: transformed row t (t < nc = rows / 2^R)
// lies in coset c (cstart[c] <= t < cstart[c + 1], cosets = the octants with
// the reflected sign bits clear); under sign pattern i it is canonical row
// t + off[c][i].
struct OctMap {
  int R, nc, ncos;
  int cstart[9];
  int off[8][8];
};
// C = M U for a scatter matrix M with the octant reflection structure, via
// its 2^R Walsh-Hadamard blocks Bh ([2^R][nc][ldb], the factor 2^-R folded
// in; ldb >= nc a multiple of 4, zero-padded); same epilogue as
// launch_gemm.  U, C: [2^R nc][N].
template <typename T>
void launch_gemm_oct(const T *Bh, int ldb, const T *U, T *C, const OctMap &om, int N, hipStream_t st,
                     const T *bias = nullptr, const double *colscale = nullptr, int cell = 8,
                     const int *pos = nullptr, const OrdInfo *rord = nullptr);
// FP32 C = A B with split-BF16 operands (three BF16 MFMA products, FP32
// accumulate); same epilogue as launch_gemm.  Asplit: A split once by
// launch_split_rows into [hi | lo][M][split_rows_kp(K)] BF16 (device,
// 2 M split_rows_kp(K) elements of 2 bytes).
int split_rows_kp(int K);
void launch_split_rows(const float *A, int M, int K, void *out, hipStream_t st);
void launch_gemm_bf16x3(const void *Asplit, const float *B, float *C, int M, int N, int K, hipStream_t st,
                        const float *bias = nullptr, const double *colscale = nullptr, int cell = 8,
                        const int *pos = nullptr, const OrdInfo *rord = nullptr);
// Octant-group product (as launch_gemm_oct) with split-BF16 operands: Bsplit
// holds the blocks Bh ([2^R nc][ldb], FP32) split by launch_split_rows with
// K = ldb, row stride kp = split_rows_kp(ldb).
void launch_gemm_oct_bf16x3(const void *Bsplit, int kp, const float *U, float *C, const OctMap &om, int N,
                            hipStream_t st, const float *bias = nullptr, const double *colscale = nullptr,
                            int cell = 8, const int *pos = nullptr, const OrdInfo *rord = nullptr);

}  // namespace tr
