// Scatter-source GEMM on the CDNA4 matrix cores.
//
// The scatter source of Section 5.2 is, for every spatial dof, a product of
// the dense angular matrix (A x A: X diag(f_n) X^T, or its ordinate-form
// image) with the vector of angular values at that dof.  With vectors laid
// out [angular][spatial] this is one GEMM  C[A][S] = G[A][A] * U[A][S]  with
// a very long N = S dimension.
//
// Tiling: a 256-thread workgroup (4 wave64s, 2 x 2) computes a BM x BN tile
// of C; A and B slices of depth BK are staged through two LDS buffers
// k-major, the next slice being loaded into registers (16-byte vector loads)
// and stored into the idle buffer while the current one feeds the MFMAs
// (one workgroup barrier per slice).  Each wave issues 16x16x4 MFMAs: lane l
// supplies A[l%16][k0 + l/16] and B[k0 + l/16][l%16]; accumulator element r
// of lane l is D[row][l%16] with row = 4 (l/16) + r for the FP32
// instruction and row = l/16 + 4 r for the FP64 one (checked on gfx950).
//
// Tile order: workgroups are dispatched round-robin over the 8 XCDs, each
// with its own L2.  Workgroup b runs on XCD b % 8; the tiles are assigned so
// that every M block of one N block (which all read the same B tile) runs on
// the same XCD, one after another, and B is fetched from HBM about once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>

#include "internal.h"

namespace tr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;

template <>
struct Mma<double> {
  using acc_t = d4;
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mma<float> {
  using acc_t = f4;
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// 16-byte vector of T
template <typename T>
struct Vec16 {
  static constexpr int n = 16 / sizeof(T);
  T v[n];
};

constexpr int kXcds = 8;

// Spatial dofs per cell (4 or 8, checked at launch) as a shift: the
// epilogues' column -> cell arithmetic without integer division.
__device__ __forceinline__ int cell_shift(int cell) { return cell == 8 ? 3 : 2; }

// Plane-layout output (a sweep input): column gn of row gm goes to the
// cell's position in row gm's orientation list, keeping the node index; the
// bias is read at the same place.  The workgroup stages the orientation of
// its rows and the positions of its columns' cells (all 8 orientations) in
// LDS once, so the epilogue takes no dependent global loads.
template <int BM, int BN>
struct OutMap {
  unsigned char flip[BM];
  int pos[8][BN / 4];  // cells of the tile (a cell spans >= 4 columns)
};

template <int BM, int BN>
__device__ __forceinline__ void out_map_load(OutMap<BM, BN> &om, const int *pos, const OrdInfo *rord, int m0,
                                             long long n0, int M, int N, int cell) {
  const long long C = N / cell;
  const long long c0 = n0 / cell;
  const int ncell = BN / cell;
  for (int t = threadIdx.x; t < BM + 8 * ncell; t += blockDim.x) {
    if (t < BM) {
      om.flip[t] = (unsigned char)rord[min(m0 + t, M - 1)].flip;
    } else {
      const int u = t - BM, fl = u / ncell, c = u % ncell;
      om.pos[fl][c] = pos[(long long)fl * C + min(c0 + c, C - 1)];
    }
  }
}

template <int BM, int BN>
__device__ __forceinline__ long long out_col(const OutMap<BM, BN> &om, long long gn, int gm, int m0, long long n0,
                                             int cell, const int *pos) {
  if (!pos) return gn;
  const int c = (int)(gn - n0) >> cell_shift(cell);
  return (long long)om.pos[om.flip[gm - m0]][c] * cell + (gn & (cell - 1));
}

// C = G * U, optionally C = bias + diag-per-column(colscale) * (G * U) where
// colscale[c / cell] scales column c (cell = spatial dofs per cell); bias has
// C's layout.
template <typename T, int BM, int BN, int BK, bool DB, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_gemm(
    const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ C,
                                              int M, int N, int K, int mblocks, int nblocks,
                                              const T *__restrict__ bias, const double *__restrict__ colscale,
                                              int cell, const int *__restrict__ pos,
                                              const OrdInfo *__restrict__ rord) {
  using acc_t = typename Mma<T>::acc_t;
  using V = Vec16<T>;
  constexpr int VN = V::n;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int PAD = 2;
  // per-thread vectors of the A (BM x BK) and B (BK x BN) slices
  constexpr int AVT = BM * BK / VN, BVT = BK * BN / VN;  // vectors per slice
  constexpr int AV = (AVT + 255) / 256, BV = (BVT + 255) / 256;
  constexpr int NB = DB ? 2 : 1;
  __shared__ T As[NB][BK][BM + PAD];
  __shared__ T Bs[NB][BK][BN + PAD];
  __shared__ OutMap<BM, BN> om;

  // XCD-aware tile order (see the file comment)
  const int b = blockIdx.x;
  const int xcd = b % kXcds, slot = b / kXcds;
  const int mb = slot % mblocks;
  const int nb = xcd + kXcds * (slot / mblocks);
  if (nb >= nblocks) return;
  const int m0 = mb * BM;
  const long long n0 = (long long)nb * BN;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm0 = (wave & 1) * WM, wn0 = (wave >> 1) * WN;
  const int lrow = lane & 15, lk = lane >> 4;

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int jn = 0; jn < TN; ++jn) acc[i][jn] = acc_t{0, 0, 0, 0};

  V ra[AV], rb[BV];
  // A slice: vectors along k (A row-major [M][K]); B slice: along n
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < AV; ++q) {
      const int v = tid + 256 * q;
      if (AVT % 256 != 0 && v >= AVT) break;
      const int i = v / (BK / VN), kv = (v % (BK / VN)) * VN;
      const int gm = m0 + i, gk = k0 + kv;
      if (gm < M && gk + VN <= K) {
        ra[q] = *reinterpret_cast<const V *>(A + (long long)gm * K + gk);
      } else {
#pragma unroll
        for (int e = 0; e < VN; ++e) ra[q].v[e] = (gm < M && gk + e < K) ? A[(long long)gm * K + gk + e] : T(0);
      }
    }
#pragma unroll
    for (int q = 0; q < BV; ++q) {
      const int v = tid + 256 * q;
      if (BVT % 256 != 0 && v >= BVT) break;
      const int kk = v / (BN / VN), nv = (v % (BN / VN)) * VN;
      const int gk = k0 + kk;
      const long long gn = n0 + nv;
      if (gk < K && gn + VN <= N) {
        rb[q] = *reinterpret_cast<const V *>(B + (long long)gk * N + gn);
      } else {
#pragma unroll
        for (int e = 0; e < VN; ++e) rb[q].v[e] = (gk < K && gn + e < N) ? B[(long long)gk * N + gn + e] : T(0);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < AV; ++q) {
      const int v = tid + 256 * q;
      if (AVT % 256 != 0 && v >= AVT) break;
      const int i = v / (BK / VN), kv = (v % (BK / VN)) * VN;
#pragma unroll
      for (int e = 0; e < VN; ++e) As[buf][kv + e][i] = ra[q].v[e];
    }
#pragma unroll
    for (int q = 0; q < BV; ++q) {
      const int v = tid + 256 * q;
      if (BVT % 256 != 0 && v >= BVT) break;
      const int kk = v / (BN / VN), nv = (v % (BN / VN)) * VN;
#pragma unroll
      for (int e = 0; e < VN; ++e) Bs[buf][kk][nv + e] = rb[q].v[e];
    }
  };

  auto mma_slice = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      T a[TM], bb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[buf][ks + lk][wm0 + i * 16 + lrow];
#pragma unroll
      for (int jn = 0; jn < TN; ++jn) bb[jn] = Bs[buf][ks + lk][wn0 + jn * 16 + lrow];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int jn = 0; jn < TN; ++jn) acc[i][jn] = Mma<T>::op(a[i], bb[jn], acc[i][jn]);
    }
  };
  if (pos) out_map_load<BM, BN>(om, pos, rord, m0, n0, M, N, cell);  // read after the loop's barriers
  load(0);
  if (DB) {
    // double-buffered: slice k+1 is loaded into registers during the MFMAs
    // on slice k and stored into the other LDS buffer (last read one slice
    // ago); one barrier per slice
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
      const bool more = k0 + BK < K;
      if (more) load(k0 + BK);
      mma_slice(buf);
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += BK) {
      store(0);
      __syncthreads();
      if (k0 + BK < K) load(k0 + BK);  // next slice in flight during the MFMAs
      mma_slice(0);
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int jn = 0; jn < TN; ++jn) {
      const long long gn = n0 + wn0 + jn * 16 + lrow;
      const T cs = (colscale && gn < N) ? T(colscale[gn >> cell_shift(cell)]) : T(1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm0 + i * 16 + Mma<T>::row(lk, r);
        if (gm < M && gn < N) {
          const long long o = (long long)gm * N + out_col<BM, BN>(om, gn, gm, m0, n0, cell, pos);
          T y = acc[i][jn][r];
          if (colscale) y *= cs;
          if (bias) y += bias[o];
          C[o] = y;
        }
      }
    }
}

// Split-BF16 product for FP32 operands (the preconditioner's scatter when
// its accuracy suffices): every operand element is split x = x_hi + x_lo
// with x_hi = bf16(x) and x_lo = bf16(x - x_hi), and C = A_hi B_hi +
// A_hi B_lo + A_lo B_hi is accumulated in FP32 by v_mfma_f32_16x16x32_bf16
// (the dropped A_lo B_lo and the split's own rounding leave a relative
// error of about 2^-16 per product).  A (the small level matrix) is split
// once by k_split_rows into [hi | lo][M][Kp] (rows zero-padded to Kp, a
// multiple of 32) and its MFMA operands are read straight from global
// memory (L2-resident), one k-slice ahead; B is split while it is staged
// into LDS.
// Tile 128 x 128 x 32, 256 threads as 2 x 2 waves of 64 x 64 (4 x 4 MFMA
// tiles).  Lane l of an MFMA supplies A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16], i < 8, as 16-byte vectors, so B is kept
// column-major ([column][k], padded to 40 elements so that 16-byte accesses
// of consecutive columns spread over the banks).  Accumulator element r of
// lane l is D[4 (l / 16) + r][l % 16].
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned pack_bf16(__bf16 a, __bf16 b) {
  return (unsigned)__builtin_bit_cast(unsigned short, a) | ((unsigned)__builtin_bit_cast(unsigned short, b) << 16);
}
__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__global__ void k_split_rows(const float *__restrict__ A, int M, int K, int Kp, __bf16 *__restrict__ out) {
  const long long n = (long long)M * Kp;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(t / Kp), k = (int)(t - (long long)m * Kp);
    __bf16 h = (__bf16)0.f, l = (__bf16)0.f;
    if (k < K) split_bf16(A[(long long)m * K + k], h, l);
    out[t] = h;
    out[n + t] = l;
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm_bf16x3(
    const __bf16 *__restrict__ As, int Kp, const float *__restrict__ B, float *__restrict__ C, int M, int N, int K,
    int mblocks, int nblocks, const float *__restrict__ bias, const double *__restrict__ colscale, int cell,
    const int *__restrict__ pos, const OrdInfo *__restrict__ rord) {
  constexpr int BM = 128, BN = 128, BK = 32, KP = BK + 8;
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BN][KP], Bl[2][BN][KP];
  __shared__ OutMap<BM, BN> om;
  const int b = blockIdx.x;
  const int xcd = b % kXcds, slot = b / kXcds;
  const int mb = slot % mblocks;
  const int nb = xcd + kXcds * (slot / mblocks);
  if (nb >= nblocks) return;
  const int m0 = mb * BM;
  const long long n0 = (long long)nb * BN;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm0 = (wave & 1) * 64, wn0 = (wave >> 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
  const __bf16 *Alo = As + (long long)M * Kp;

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // A operands of this lane (rows past M read row M - 1; their products
  // land in rows that are not stored)
  long long arow[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) arow[i] = (long long)min(m0 + wm0 + 16 * i + lr, M - 1) * Kp + 8 * lk;
  bf8 ah[4], al[4];
  auto load_a = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ah[i] = *reinterpret_cast<const bf8 *>(As + arow[i] + k0);
      al[i] = *reinterpret_cast<const bf8 *>(Alo + arow[i] + k0);
    }
  };
  // B staging: 16 floats per thread (column t % 128, k 16 (t / 128) + i)
  float rb[16];
  const int bn = tid & 127, bk = (tid >> 7) * 16;
  auto load_b = [&](int k0) {
    const long long gn = n0 + bn;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int gk = k0 + bk + i;
      rb[i] = (gk < K && gn < N) ? B[(long long)gk * N + gn] : 0.f;
    }
  };
  auto store_b = [&](int buf) {
    unsigned hw[8], lw[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      __bf16 h0, l0, h1, l1;
      split_bf16(rb[2 * i], h0, l0);
      split_bf16(rb[2 * i + 1], h1, l1);
      hw[i] = pack_bf16(h0, h1);
      lw[i] = pack_bf16(l0, l1);
    }
    uint4 *bh = reinterpret_cast<uint4 *>(&Bh[buf][bn][bk]);
    uint4 *bl = reinterpret_cast<uint4 *>(&Bl[buf][bn][bk]);
    bh[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    bh[1] = make_uint4(hw[4], hw[5], hw[6], hw[7]);
    bl[0] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    bl[1] = make_uint4(lw[4], lw[5], lw[6], lw[7]);
  };
  auto mma = [&](int buf, const bf8 (&xh)[4], const bf8 (&xl)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf8 bh = *reinterpret_cast<const bf8 *>(&Bh[buf][wn0 + 16 * j + lr][8 * lk]);
      const bf8 bl = *reinterpret_cast<const bf8 *>(&Bl[buf][wn0 + 16 * j + lr][8 * lk]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[i], bh, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], bl, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], bh, acc[i][j], 0, 0, 0);
      }
    }
  };
  if (pos) out_map_load<BM, BN>(om, pos, rord, m0, n0, M, N, cell);  // read after the loop's barriers
  load_a(0);
  load_b(0);
  store_b(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    const bf8 ch[4] = {ah[0], ah[1], ah[2], ah[3]}, cl[4] = {al[0], al[1], al[2], al[3]};
    if (more) {
      load_a(k0 + BK);
      load_b(k0 + BK);
    }
    mma(buf, ch, cl);
    if (more) store_b(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long gn = n0 + wn0 + 16 * j + lr;
      const float cs = (colscale && gn < N) ? (float)colscale[gn >> cell_shift(cell)] : 1.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm0 + 16 * i + 4 * lk + r;
        if (gm < M && gn < N) {
          const long long o = (long long)gm * N + out_col<BM, BN>(om, gn, gm, m0, n0, cell, pos);
          float y = acc[i][j][r];
          if (colscale) y *= cs;
          if (bias) y += bias[o];
          C[o] = y;
        }
      }
    }
}

// Octant-group scatter product.  On an angular mesh that is mapped onto
// itself by the reflections through the coordinate planes of a set of axes
// (all three on uniformly refined meshes, two on meshes refined around an
// axis), with reflected patches in the same position of their octants'
// patch lists, the scatter matrix M depends on a pair of octants only
// through their sign difference: M[(f|s1, k1), (g|s2, k2)] depends on
// s1 ^ s2 (s: the reflected sign bits, f, g: the other bits, k: position in
// the octant).  Such a matrix is block-diagonalised by the Walsh-Hadamard
// transform over the 2^R sign patterns s:
//   U^[chi][t] = sum_s (-1)^{|chi & s|} U[(f|s, k)],  t = (f, k)
//   C^[chi]    = B^[chi] U^[chi]       (2^R GEMMs of size nc = A / 2^R)
//   C[(f|s,k)] = sum_chi (-1)^{|chi & s|} C^[chi][t]
// with B^[chi][t1][t2] = 2^-R sum_s (-1)^{|chi & s|} M[(f1|0,k1),(f2|s,k2)].
// That is 2 A^2 / 2^R multiply-adds per column instead of 2 A^2.  One
// kernel does all of it: a workgroup owns a BM x BN tile of transformed rows
// for every chi at once; per k-slice the loader threads fetch the 2^R
// canonical rows of each transformed index (row = t + off[c][i], c the
// coset of t, i the sign pattern in the order of its bits: computed, no
// dependent loads) and transform them in registers into the 2^R B tiles, the other threads stage the 2^R A tiles; after the k loop each
// lane holds, for its accumulator positions, the values of every chi, and
// the inverse transform is taken in registers before the store (with the
// epilogue of k_gemm).  U and C each cross HBM once.
template <int R>
__device__ __forceinline__ int oct_row(const OctMap &om, int t, int i) {
  // coset of t (cosets are runs of transformed rows), then its offset
  constexpr int NCOS = 8 >> R;
  int off = om.off[0][i];
#pragma unroll
  for (int c = 1; c < NCOS; ++c)
    if (t >= om.cstart[c]) off = om.off[c][i];
  return t + off;
}

// Plane-layout output of the octant-group products: the positions of the
// tile's cells in every orientation's list and the orientation of every
// output row, staged in LDS by the whole workgroup.
template <int R, int BM, int BN>
__device__ __forceinline__ void oct_out_stage(int (&pos_s)[8][BN / 4 + 1], unsigned char (&flip_s)[1 << R][BM],
                                              const OctMap &om, const int *pos, const OrdInfo *rord, int nc, int m0,
                                              long long n0, int cell, long long ncells) {
  const int ncell = BN / cell;
  for (int t = threadIdx.x; t < 8 * ncell; t += blockDim.x) {
    const int fl = t / ncell, c = t % ncell;
    pos_s[fl][c] = pos[(long long)fl * ncells + min(n0 / cell + c, ncells - 1)];
  }
  for (int t = threadIdx.x; t < (1 << R) * BM; t += blockDim.x) {
    const int q = t / BM, r = m0 + t % BM;
    flip_s[q][t % BM] = r < nc ? (unsigned char)rord[oct_row<R>(om, r, q)].flip : 0;
  }
}

// Output stage of the octant-group products: for each accumulator position
// (transformed row t, column) the 2^R values of the sign patterns chi are
// transformed back in registers and stored with the epilogue of k_gemm.
// Accumulator element r of lane (lrow, lk) of MFMA tile (i, jn) is row
// wm0 + 16 i + Mma<T>::row(lk, r), column wn0 + 16 jn + lrow of the tile.
template <typename T, int R, int BM, int BN, int TM, int TN>
__device__ __forceinline__ void oct_store(const typename Mma<T>::acc_t (&acc)[1 << R][TM][TN], T *__restrict__ C,
                                          const OctMap &om, int nc, int N, int m0, long long n0, int wm0, int wn0,
                                          int lrow, int lk, const T *__restrict__ bias,
                                          const double *__restrict__ colscale, int cell, const int *pos,
                                          const int (&pos_s)[8][BN / 4 + 1],
                                          const unsigned char (&flip_s)[1 << R][BM]) {
  constexpr int NCHI = 1 << R;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int jn = 0; jn < TN; ++jn) {
      const long long gn = n0 + wn0 + jn * 16 + lrow;
      const T cs = (colscale && gn < N) ? T(colscale[gn >> cell_shift(cell)]) : T(1);
      const int cl = (int)(gn - n0) >> cell_shift(cell), within = (int)(gn & (cell - 1));
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = m0 + wm0 + i * 16 + Mma<T>::row(lk, r);
        if (t >= nc || gn >= N) continue;
        T y[NCHI];
#pragma unroll
        for (int j = 0; j < NCHI; ++j) y[j] = acc[j][i][jn][r];
#pragma unroll
        for (int hh = 1; hh < NCHI; hh <<= 1)
#pragma unroll
          for (int q = 0; q < NCHI; ++q)
            if (!(q & hh)) {
              const T a = y[q], c = y[q + hh];
              y[q] = a + c;
              y[q + hh] = a - c;
            }
#pragma unroll
        for (int q = 0; q < NCHI; ++q) {
          const long long row = oct_row<R>(om, t, q);
          long long col = gn;
          if (pos) col = (long long)pos_s[flip_s[q][t - m0]][cl] * cell + within;
          const long long o = row * N + col;
          T v = y[q];
          if (colscale) v *= cs;
          if (bias) v += bias[o];
          C[o] = v;
        }
      }
    }
}

template <typename T, int R, int BM, int BN, int BK, int WPE, bool DB, bool ALL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_gemm_oct(
    const T *__restrict__ Bh, int ldb, const T *__restrict__ U, T *__restrict__ C, OctMap om, int nc, int N,
    int mblocks, int nblocks, const T *__restrict__ bias, const double *__restrict__ colscale, int cell,
    const int *__restrict__ pos, const OrdInfo *__restrict__ rord, long long ncells) {
  constexpr int NCHI = 1 << R;
  using acc_t = typename Mma<T>::acc_t;
  using V = Vec16<T>;
  constexpr int VN = V::n;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int PAD = 2;
  // U loader threads: one (k, column vector) each; the A tiles are staged
  // by the other threads, or (ALL) by every thread
  constexpr int BPAIRS = BK * BN / VN;
  constexpr int ATHREADS = ALL ? 256 : 256 - BPAIRS;
  constexpr int AVT = NCHI * BM * BK / VN;         // A vectors per slice
  constexpr int AV = (AVT + ATHREADS - 1) / ATHREADS;
  static_assert(BK % 4 == 0 && BK % VN == 0 && BPAIRS <= (ALL ? 256 : 128), "tile shape");
  constexpr int NBUF = DB ? 2 : 1;
  __shared__ T As[NBUF][NCHI][BK][BM + PAD];
  __shared__ T Bs[NBUF][NCHI][BK][BN + PAD];
  __shared__ int pos_s[8][BN / 4 + 1];
  __shared__ unsigned char flip_s[NCHI][BM];  // orientation of each output row (plane layout)

  const int b = blockIdx.x;
  const int xcd = b % kXcds, slot = b / kXcds;
  const int mb = slot % mblocks;
  const int nb = xcd + kXcds * (slot / mblocks);
  if (nb >= nblocks) return;
  const int m0 = mb * BM;
  const long long n0 = (long long)nb * BN;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm0 = (wave & 1) * WM, wn0 = (wave >> 1) * WN;
  const int lrow = lane & 15, lk = lane >> 4;

  acc_t acc[NCHI][TM][TN];
#pragma unroll
  for (int j = 0; j < NCHI; ++j)
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int jn = 0; jn < TN; ++jn) acc[j][i][jn] = acc_t{0, 0, 0, 0};

  V rx[NCHI];   // U rows of one (k, column vector), loader threads
  V ra[AV];     // A vectors, staging threads
  const bool loader = tid < BPAIRS;
  const bool aload = ALL || !loader;
  const int bk = tid / (BN / VN), bnv = (tid % (BN / VN)) * VN;
  auto load = [&](int k0) {
    if (loader) {
      const int gk = k0 + bk;
      const long long gn = n0 + bnv;
#pragma unroll
      for (int i = 0; i < NCHI; ++i) {
        if (gk < nc) {
          const long long row = oct_row<R>(om, gk, i);
          if (gn + VN <= N) {
            rx[i] = *reinterpret_cast<const V *>(U + row * N + gn);
          } else {
#pragma unroll
            for (int e = 0; e < VN; ++e) rx[i].v[e] = gn + e < N ? U[row * N + gn + e] : T(0);
          }
        } else {
#pragma unroll
          for (int e = 0; e < VN; ++e) rx[i].v[e] = T(0);
        }
      }
    }
    if (aload) {
      const int idx = ALL ? tid : tid - BPAIRS;
#pragma unroll
      for (int q = 0; q < AV; ++q) {
        const int v = idx + ATHREADS * q;
        if (AVT % ATHREADS != 0 && v >= AVT) break;
        const int j = v / (BM * BK / VN), rem = v % (BM * BK / VN);
        const int i = rem / (BK / VN), kv = (rem % (BK / VN)) * VN;
        const int gm = m0 + i, gk = k0 + kv;
        if (gm < nc && gk < ldb) {
          ra[q] = *reinterpret_cast<const V *>(Bh + ((long long)j * nc + gm) * ldb + gk);
        } else {
#pragma unroll
          for (int e = 0; e < VN; ++e) ra[q].v[e] = T(0);
        }
      }
    }
  };
  auto store = [&](int buf) {
    if (loader) {
      // forward transform over the sign patterns, in registers
#pragma unroll
      for (int hh = 1; hh < NCHI; hh <<= 1)
#pragma unroll
        for (int i = 0; i < NCHI; ++i)
          if (!(i & hh)) {
#pragma unroll
            for (int e = 0; e < VN; ++e) {
              const T a = rx[i].v[e], c = rx[i + hh].v[e];
              rx[i].v[e] = a + c;
              rx[i + hh].v[e] = a - c;
            }
          }
#pragma unroll
      for (int j = 0; j < NCHI; ++j)
#pragma unroll
        for (int e = 0; e < VN; ++e) Bs[buf][j][bk][bnv + e] = rx[j].v[e];
    }
    if (aload) {
      const int idx = ALL ? tid : tid - BPAIRS;
#pragma unroll
      for (int q = 0; q < AV; ++q) {
        const int v = idx + ATHREADS * q;
        if (AVT % ATHREADS != 0 && v >= AVT) break;
        const int j = v / (BM * BK / VN), rem = v % (BM * BK / VN);
        const int i = rem / (BK / VN), kv = (rem % (BK / VN)) * VN;
#pragma unroll
        for (int e = 0; e < VN; ++e) As[buf][j][kv + e][i] = ra[q].v[e];
      }
    }
  };
  auto mma_slice = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
#pragma unroll
      for (int j = 0; j < NCHI; ++j) {
        T a[TM], bb[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[buf][j][ks + lk][wm0 + i * 16 + lrow];
#pragma unroll
        for (int jn = 0; jn < TN; ++jn) bb[jn] = Bs[buf][j][ks + lk][wn0 + jn * 16 + lrow];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int jn = 0; jn < TN; ++jn) acc[j][i][jn] = Mma<T>::op(a[i], bb[jn], acc[j][i][jn]);
      }
    }
  };
  if (pos) oct_out_stage<R, BM, BN>(pos_s, flip_s, om, pos, rord, nc, m0, n0, cell, ncells);  // read after the loop's barriers
  // DB: two LDS buffers, the next slice stored during the MFMAs, one
  // barrier per slice; else one buffer, the next slice's loads in flight
  // during the MFMAs, two barriers per slice
  load(0);
  if (DB) {
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < nc; k0 += BK) {
      const bool more = k0 + BK < nc;
      if (more) load(k0 + BK);
      mma_slice(buf);
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  } else {
    for (int k0 = 0; k0 < nc; k0 += BK) {
      store(0);
      __syncthreads();
      if (k0 + BK < nc) load(k0 + BK);
      mma_slice(0);
      __syncthreads();
    }
  }
  oct_store<T, R, BM, BN, TM, TN>(acc, C, om, nc, N, m0, n0, wm0, wn0, lrow, lk, bias, colscale, cell, pos, pos_s,
                                  flip_s);
}

// Split-BF16 form of the octant-group product (FP32 operands: the
// preconditioner's scatter when its accuracy suffices).  The blocks B^[chi]
// are split once by k_split_rows ([hi | lo][2^R nc][kp]) and their MFMA
// operands read straight from global memory (L2-resident), one sign pattern
// ahead; per k-slice of 32 every thread loads, for one column and 8
// transformed rows k, the 2^R canonical rows of each k, transforms them over
// the sign patterns in FP32, splits each value x = bf16(x) + bf16(x -
// bf16(x)) and stores both parts in LDS column-major ([chi][column][k]), as
// 16-byte chunks of 8 k whose chunk index is XOR-swizzled with bits 1-2 of
// the column: the 16-byte reads and writes of 8 consecutive columns then
// cover all banks.  Each product is three v_mfma_f32_16x16x32_bf16 (lo hi,
// hi lo, hi hi), FP32 accumulate, the relative error of k_gemm_bf16x3.
// Tile BM x 64 for every chi, 2 x 2 waves; the output stage of k_gemm_oct.
template <int R, int BM, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_gemm_oct_bf16x3(
    const __bf16 *__restrict__ Bs, int kp, const float *__restrict__ U, float *__restrict__ C, OctMap om, int nc,
    int N, int mblocks, int nblocks, const float *__restrict__ bias, const double *__restrict__ colscale, int cell,
    const int *__restrict__ pos, const OrdInfo *__restrict__ rord, long long ncells) {
  constexpr int NCHI = 1 << R;
  constexpr int BN = 64, BK = 32, KG = 8;  // KG: k values per thread (64 columns x 4 groups)
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert(BM % 32 == 0 && 256 / BN * KG == BK, "tile shape");
  __shared__ __attribute__((aligned(16))) __bf16 Bhi[NCHI][BN][BK], Blo[NCHI][BN][BK];
  __shared__ int pos_s[8][BN / 4 + 1];
  __shared__ unsigned char flip_s[NCHI][BM];

  const int b = blockIdx.x;
  const int xcd = b % kXcds, slot = b / kXcds;
  const int mb = slot % mblocks;
  const int nb = xcd + kXcds * (slot / mblocks);
  if (nb >= nblocks) return;
  const int m0 = mb * BM;
  const long long n0 = (long long)nb * BN;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm0 = (wave & 1) * WM, wn0 = (wave >> 1) * WN;
  const int lrow = lane & 15, lk = lane >> 4;
  const __bf16 *Bl = Bs + (long long)NCHI * nc * kp;

  f4 acc[NCHI][TM][TN];
#pragma unroll
  for (int j = 0; j < NCHI; ++j)
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int jn = 0; jn < TN; ++jn) acc[j][i][jn] = f4{0.f, 0.f, 0.f, 0.f};

  // staging: column c, transformed rows k0 + KG g .. + KG - 1
  const int c = tid % BN, g = tid / BN;
  const long long gn = n0 + c;
  const bool col_ok = gn < N;
  float rx[KG][NCHI];
  auto load = [&](int k0) {
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
      const int k = k0 + KG * g + kk;
#pragma unroll
      for (int i = 0; i < NCHI; ++i)
        rx[kk][i] = (k < nc && col_ok) ? U[(long long)oct_row<R>(om, k, i) * N + gn] : 0.f;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
      for (int hh = 1; hh < NCHI; hh <<= 1)
#pragma unroll
        for (int i = 0; i < NCHI; ++i)
          if (!(i & hh)) {
            const float a = rx[kk][i], d = rx[kk][i + hh];
            rx[kk][i] = a + d;
            rx[kk][i + hh] = a - d;
          }
    const int ch = g ^ ((c >> 1) & 3);
#pragma unroll
    for (int j = 0; j < NCHI; ++j) {
      unsigned hw[KG / 2], lw[KG / 2];
#pragma unroll
      for (int e = 0; e < KG / 2; ++e) {
        __bf16 h0, l0, h1, l1;
        split_bf16(rx[2 * e][j], h0, l0);
        split_bf16(rx[2 * e + 1][j], h1, l1);
        hw[e] = pack_bf16(h0, h1);
        lw[e] = pack_bf16(l0, l1);
      }
      *reinterpret_cast<uint4 *>(&Bhi[j][c][8 * ch]) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      *reinterpret_cast<uint4 *>(&Blo[j][c][8 * ch]) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
  };
  // A operand rows of this lane (rows past nc read row nc - 1 of the same
  // block: their products land in rows that are not stored)
  long long arow[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) arow[i] = (long long)min(m0 + wm0 + 16 * i + lrow, nc - 1) * kp + 8 * lk;
  auto mma = [&](int k0) {
    bf8 ah[2][TM], al[2][TM];
    auto load_a = [&](int j, int sl) {
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const long long o = (long long)j * nc * kp + arow[i] + k0;
        ah[sl][i] = *reinterpret_cast<const bf8 *>(Bs + o);
        al[sl][i] = *reinterpret_cast<const bf8 *>(Bl + o);
      }
    };
    load_a(0, 0);
#pragma unroll
    for (int j = 0; j < NCHI; ++j) {
      if (j + 1 < NCHI) load_a(j + 1, (j + 1) & 1);
      bf8 bh[TN], bl[TN];
#pragma unroll
      for (int jn = 0; jn < TN; ++jn) {
        const int col = wn0 + 16 * jn + lrow;
        const int chk = lk ^ ((col >> 1) & 3);
        bh[jn] = *reinterpret_cast<const bf8 *>(&Bhi[j][col][8 * chk]);
        bl[jn] = *reinterpret_cast<const bf8 *>(&Blo[j][col][8 * chk]);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int jn = 0; jn < TN; ++jn) {
          f4 a = acc[j][i][jn];
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[j & 1][i], bh[jn], a, 0, 0, 0);
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[j & 1][i], bl[jn], a, 0, 0, 0);
          acc[j][i][jn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[j & 1][i], bh[jn], a, 0, 0, 0);
        }
    }
  };
  if (pos) oct_out_stage<R, BM, BN>(pos_s, flip_s, om, pos, rord, nc, m0, n0, cell, ncells);  // read after the loop's barriers
  // one LDS buffer: the next slice's loads in flight during the MFMAs, two
  // barriers per slice
  load(0);
  for (int k0 = 0; k0 < nc; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < nc) load(k0 + BK);
    mma(k0);
    __syncthreads();
  }
  oct_store<float, R, BM, BN, TM, TN>(acc, C, om, nc, N, m0, n0, wm0, wn0, lrow, lk, bias, colscale, cell, pos,
                                      pos_s, flip_s);
}

}  // namespace

// Launch shapes (tile M x N x depth, LDS double buffering, minimum waves per
// SIMD the register allocation must allow), chosen by measurement on MI355X
// (32^3 problem, A = 384 and 1104): FP64 64 x 128 x 8 with four waves per
// SIMD (53-57 TF/s), FP32 128 x 128 x 16 (108-110 TF/s).
template <typename T, int BM, int BN, int BK, bool DB, int WPE>
static void launch_shape(const T *A, const T *B, T *C, int M, int N, int K, hipStream_t st, const T *bias,
                         const double *colscale, int cell, const int *pos, const OrdInfo *rord) {
  const int mblocks = (M + BM - 1) / BM;
  const int nblocks = (int)(((long long)N + BN - 1) / BN);
  const long long nb_pad = ((long long)nblocks + kXcds - 1) / kXcds * kXcds;
  const long long grid = (long long)mblocks * nb_pad;
  hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, DB, WPE>), dim3((unsigned)grid), dim3(256), 0, st, A, B, C, M, N, K,
                     mblocks, nblocks, bias, colscale, cell, pos, rord);
}

template <typename T>
void launch_gemm(const T *A, const T *B, T *C, int M, int N, int K, hipStream_t st, const T *bias,
                 const double *colscale, int cell, const int *pos, const OrdInfo *rord) {
  if ((cell != 4 && cell != 8) || (pos && !rord)) throw std::runtime_error("GEMM: bad epilogue arguments");
  if (sizeof(T) == 8)
    launch_shape<T, 64, 128, 8, true, 4>(A, B, C, M, N, K, st, bias, colscale, cell, pos, rord);
  else
    launch_shape<T, 128, 128, 16, true, 0>(A, B, C, M, N, K, st, bias, colscale, cell, pos, rord);
}
// Octant-group product (see k_gemm_oct): 256 threads, LDS double buffering.
template <typename T, int R, int BM, int BN, int BK, int WPE, bool DB, bool ALL>
static void launch_oct_shape(const T *Bh, int ldb, const T *U, T *C, const OctMap &om, int nc, int N, hipStream_t st,
                             const T *bias, const double *colscale, int cell, const int *pos, const OrdInfo *rord) {
  const int mblocks = (nc + BM - 1) / BM;
  const int nblocks = (int)(((long long)N + BN - 1) / BN);
  const long long nb_pad = ((long long)nblocks + kXcds - 1) / kXcds * kXcds;
  const long long grid = (long long)mblocks * nb_pad;
  hipLaunchKernelGGL((k_gemm_oct<T, R, BM, BN, BK, WPE, DB, ALL>), dim3((unsigned)grid), dim3(256), 0, st, Bh, ldb, U, C, om,
                     nc, N, mblocks, nblocks, bias, colscale, cell, pos, rord, (long long)(N / cell));
}

template <typename T>
void launch_gemm_oct(const T *Bh, int ldb, const T *U, T *C, const OctMap &om, int N, hipStream_t st, const T *bias,
                     const double *colscale, int cell, const int *pos, const OrdInfo *rord) {
  if ((cell != 4 && cell != 8) || (pos && !rord)) throw std::runtime_error("octant-group GEMM: bad epilogue arguments");
  const int nc = om.nc;
#define TR_OCT(BM, BN, BK, WPE, DB, ALL)                                                                              \
  switch (om.R) {                                                                                                 \
    case 1:                                                                                                       \
      launch_oct_shape<T, 1, BM, BN, BK, WPE, DB, ALL>(Bh, ldb, U, C, om, nc, N, st, bias, colscale, cell, pos, rord); \
      break;                                                                                                      \
    case 2:                                                                                                       \
      launch_oct_shape<T, 2, BM, BN, BK, WPE, DB, ALL>(Bh, ldb, U, C, om, nc, N, st, bias, colscale, cell, pos, rord); \
      break;                                                                                                      \
    case 3:                                                                                                       \
      launch_oct_shape<T, 3, BM, BN, BK, WPE, DB, ALL>(Bh, ldb, U, C, om, nc, N, st, bias, colscale, cell, pos, rord); \
      break;                                                                                                      \
    default: throw std::runtime_error("octant-group GEMM: 1 to 3 reflected axes");                                \
  }
  // shapes measured on MI355X (three axes, N = 884736): FP64 32 x 64 x 8
  // with one LDS buffer and every thread loading, two waves per SIMD, 15.2
  // ms at nc = 192 (34 TF/s) and 2.0 ms at nc = 48 (32 x 32 x 8 and 16: 19
  // and 17 ms); FP32 32 x 64 x 16 with one LDS buffer, every thread
  // loading, three waves per SIMD, 8.2 and 1.16 ms (32 x 64 x 8 double
  // buffered: 9.1 and 1.3 ms; 64 x 64 x 16: 8.3 and 1.5 ms)
  if constexpr (sizeof(T) == 8) {
    TR_OCT(32, 64, 8, 2, false, true)
  } else {
    TR_OCT(32, 64, 16, 3, false, true)
  }
#undef TR_OCT
}
template void launch_gemm_oct<double>(const double *, int, const double *, double *, const OctMap &, int,
                                      hipStream_t, const double *, const double *, int, const int *,
                                      const OrdInfo *);
template void launch_gemm_oct<float>(const float *, int, const float *, float *, const OctMap &, int, hipStream_t,
                                     const float *, const double *, int, const int *, const OrdInfo *);

int split_rows_kp(int K) { return (K + 31) / 32 * 32; }

void launch_split_rows(const float *A, int M, int K, void *out, hipStream_t st) {
  const int Kp = split_rows_kp(K);
  const long long n = (long long)M * Kp;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_split_rows, dim3(blocks), dim3(256), 0, st, A, M, K, Kp, reinterpret_cast<__bf16 *>(out));
}

void launch_gemm_bf16x3(const void *Asplit, const float *B, float *C, int M, int N, int K, hipStream_t st,
                        const float *bias, const double *colscale, int cell, const int *pos, const OrdInfo *rord) {
  if ((cell != 4 && cell != 8) || (pos && !rord)) throw std::runtime_error("GEMM: bad epilogue arguments");
  const int mblocks = (M + 127) / 128;
  const int nblocks = (int)(((long long)N + 127) / 128);
  const long long nb_pad = ((long long)nblocks + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(k_gemm_bf16x3, dim3((unsigned)(mblocks * nb_pad)), dim3(256), 0, st,
                     reinterpret_cast<const __bf16 *>(Asplit), split_rows_kp(K), B, C, M, N, K, mblocks, nblocks,
                     bias, colscale, cell, pos, rord);
}

template <int R, int BM, int WPE>
static void launch_oct_bf16_shape(const __bf16 *Bs, int kp, const float *U, float *C, const OctMap &om, int N,
                                  hipStream_t st, const float *bias, const double *colscale, int cell, const int *pos,
                                  const OrdInfo *rord) {
  const int nc = om.nc;
  const int mblocks = (nc + BM - 1) / BM;
  const int nblocks = (int)(((long long)N + 63) / 64);
  const long long nb_pad = ((long long)nblocks + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL((k_gemm_oct_bf16x3<R, BM, WPE>), dim3((unsigned)(mblocks * nb_pad)), dim3(256), 0, st, Bs, kp, U,
                     C, om, nc, N, mblocks, nblocks, bias, colscale, cell, pos, rord, (long long)(N / cell));
}

void launch_gemm_oct_bf16x3(const void *Bsplit, int kp, const float *U, float *C, const OctMap &om, int N,
                            hipStream_t st, const float *bias, const double *colscale, int cell, const int *pos,
                            const OrdInfo *rord) {
  if ((cell != 4 && cell != 8) || (pos && !rord)) throw std::runtime_error("octant-group GEMM: bad epilogue arguments");
  if (kp % 32 != 0 || kp < om.nc) throw std::runtime_error("octant-group GEMM: bad split block stride");
  const __bf16 *Bs = reinterpret_cast<const __bf16 *>(Bsplit);
  // tile 32 x 64 x 32, two waves per SIMD: measured on MI355X (three axes,
  // N = 884736) 9.1 ms at nc = 192 and 1.55 ms at nc = 48, the times of the
  // FP32 product (9.3 and 1.3-1.6 ms): both are bound by the latency of the
  // operand loads, not by the matrix cores (64 x 64 tiles at one wave per
  // SIMD: 13 and 2.7 ms; the A operands of a slice loaded ahead of the next
  // slice's U loads: no change)
  switch (om.R) {
    case 1: launch_oct_bf16_shape<1, 32, 2>(Bs, kp, U, C, om, N, st, bias, colscale, cell, pos, rord); break;
    case 2: launch_oct_bf16_shape<2, 32, 2>(Bs, kp, U, C, om, N, st, bias, colscale, cell, pos, rord); break;
    case 3: launch_oct_bf16_shape<3, 32, 2>(Bs, kp, U, C, om, N, st, bias, colscale, cell, pos, rord); break;
    default: throw std::runtime_error("octant-group GEMM: 1 to 3 reflected axes");
  }
}

template void launch_gemm<double>(const double *, const double *, double *, int, int, int, hipStream_t,
                                  const double *, const double *, int, const int *, const OrdInfo *);
template void launch_gemm<float>(const float *, const float *, float *, int, int, int, hipStream_t, const float *,
                                 const double *, int, const int *, const OrdInfo *);

}  // namespace tr
