// Scatter-source GEMM on the CDNA4 matrix cores.
//
// The scatter source of Section 5.2 is, for every spatial dof, a product of
// the dense angular matrix (A x A: X diag(f_n) X^T, or its ordinate-form
// image) with the vector of angular values at that dof.  With vectors laid
// out [angular][spatial] this is one GEMM  C[A][S] = G[A][A] * U[A][S]  with
// a very long N = S dimension.
//
// Tiling: a 256-thread workgroup (4 wave64s, 2 x 2) computes a BM x BN tile
// of C; A and B tiles of depth BK are staged through LDS k-major, and each
// wave issues 16x16x4 MFMAs: lane l supplies A[l%16][k0 + l/16] and
// B[k0 + l/16][l%16]; accumulator element r of lane l is D[row][l%16] with
// row = 4 (l/16) + r for the FP32 instruction and row = l/16 + 4 r for the
// FP64 one (checked on gfx950).
// Workgroup ids run over M fastest so the workgroups that share a B tile
// (an N block) are dispatched together and hit it in L2.
#include <hip/hip_runtime.h>

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

template <typename T, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void k_gemm(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ C,
                                              int M, int N, int K, int mblocks) {
  using acc_t = typename Mma<T>::acc_t;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int PAD = 4;
  __shared__ T As[BK][BM + PAD];
  __shared__ T Bs[BK][BN + PAD];

  const int bid = blockIdx.x;
  const int mb = bid % mblocks, nb = bid / mblocks;
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

  for (int k0 = 0; k0 < K; k0 += BK) {
    // stage A[m0:m0+BM][k0:k0+BK] as As[k][m]
#pragma unroll
    for (int e = tid; e < BM * BK; e += 256) {
      const int kk = e % BK, i = e / BK;
      const int gm = m0 + i, gk = k0 + kk;
      As[kk][i] = (gm < M && gk < K) ? A[(long long)gm * K + gk] : T(0);
    }
    // stage B[k0:k0+BK][n0:n0+BN] as Bs[k][n]
#pragma unroll
    for (int e = tid; e < BN * BK; e += 256) {
      const int jn = e % BN, kk = e / BN;
      const int gk = k0 + kk;
      const long long gn = n0 + jn;
      Bs[kk][jn] = (gk < K && gn < N) ? B[(long long)gk * N + gn] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      T a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[ks + lk][wm0 + i * 16 + lrow];
#pragma unroll
      for (int jn = 0; jn < TN; ++jn) b[jn] = Bs[ks + lk][wn0 + jn * 16 + lrow];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int jn = 0; jn < TN; ++jn) acc[i][jn] = Mma<T>::op(a[i], b[jn], acc[i][jn]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int jn = 0; jn < TN; ++jn) {
      const long long gn = n0 + wn0 + jn * 16 + lrow;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm0 + i * 16 + Mma<T>::row(lk, r);
        if (gm < M && gn < N) C[(long long)gm * N + gn] = acc[i][jn][r];
      }
    }
}

}  // namespace

template <typename T>
void launch_gemm(const T *A, const T *B, T *C, int M, int N, int K, hipStream_t st) {
  constexpr int BM = 64, BN = 64, BK = 16;
  const int mblocks = (M + BM - 1) / BM;
  const long long nblocks = ((long long)N + BN - 1) / BN;
  const long long grid = mblocks * nblocks;
  hipLaunchKernelGGL((k_gemm<T, BM, BN, BK>), dim3((unsigned)grid), dim3(256), 0, st, A, B, C, M, N, K, mblocks);
}
template void launch_gemm<double>(const double *, const double *, double *, int, int, int, hipStream_t);
template void launch_gemm<float>(const float *, const float *, float *, int, int, int, hipStream_t);

}  // namespace tr
