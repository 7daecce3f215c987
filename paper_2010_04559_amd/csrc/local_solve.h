// Per-cell, per-ordinate DG transport block solve.
//
// With the collocated 3-point angular rule every (cell, patch) block of the
// weak form (eq. complete) splits into one system per ordinate Omega_k
// after the fixed change of basis u_k = sum_d psi_d(Omega_k) phi_d.  For an
// ordinate with a_xi = |Omega_k,xi| and c_xi = a_xi / h_xi, in coordinates
// oriented along the flow (node 0 upstream on every axis), the cell matrix
// of the nodal Q1 upwind DG discretisation is
//     A = N (sum_xi c_xi E_xi + sigma I),   E = [[3, 1], [-3, 1]] on axis xi,
// N the cell mass matrix.  E has eigenvalues 2 +- i sqrt(2) and all E_xi
// commute, so A^{-1} N = (V (x) V (x) V) D^{-1} (V (x) V (x) V)^{-1} with
// D_mu = sigma + sum_xi c_xi lambda_{mu_xi}: four (3-D) or two (2-D)
// complex scalings after tensor-product 2x2 transforms.  Modes come in
// conjugate pairs, so only those with mu_x = + are formed.
//
// The transposed block (adjoint sweep) uses A^T = (sum c E_xi^T + sigma) N,
// whose transforms are V^T forward and V^{-T} back.
#pragma once

#if defined(__HIPCC__)
#define TR_HD __host__ __device__ __forceinline__
#else
#define TR_HD inline
#endif

namespace tr {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
TR_HD cx<T> cmul(cx<T> a, cx<T> b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
template <typename T>
TR_HD cx<T> cmulc(cx<T> a, cx<T> b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }  // conj(a)*b
template <typename T>
TR_HD cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
TR_HD cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
TR_HD cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
TR_HD cx<T> cinv(cx<T> a) {
  T r = T(1) / (a.re * a.re + a.im * a.im);
  return {a.re * r, -a.im * r};
}

// Mode-(+) transform coefficients of one axis in physical node order.
//   fwd[b]: contribution of node value b to mode +
//   bwd[b]: contribution of mode + to node value b (mode - is the conjugate)
template <typename T>
struct AxisXf {
  cx<T> fwd[2], bwd[2];
};

template <typename T>
TR_HD AxisXf<T> axis_xf(bool flip, bool transpose) {
  const T q = T(0.35355339059327376220);  // 1 / (2 sqrt 2)
  const T r2 = T(1.41421356237309504880);
  // oriented: V^{-1}[+,0] = 1/2 - i q, V^{-1}[+,1] = -i q; V[0,+] = 1, V[1,+] = -1 + i sqrt 2
  cx<T> r0{T(0.5), -q}, r1{T(0), -q}, v0{T(1), T(0)}, v1{T(-1), r2};
  AxisXf<T> a;
  cx<T> f0 = transpose ? v0 : r0, f1 = transpose ? v1 : r1;
  cx<T> b0 = transpose ? r0 : v0, b1 = transpose ? r1 : v1;
  a.fwd[0] = flip ? f1 : f0;
  a.fwd[1] = flip ? f0 : f1;
  a.bwd[0] = flip ? b1 : b0;
  a.bwd[1] = flip ? b0 : b1;
  return a;
}

template <typename T>
TR_HD cx<T> rmul(cx<T> a, T x) { return {a.re * x, a.im * x}; }

// Forward transform of one real nodal vector into the mu_x = + modes.
// 3-D: out[my*2 + mz] (my, mz: 0 = +, 1 = -); 2-D: out[my].
template <typename T, int DIM>
TR_HD void modes_forward(const T *v, const AxisXf<T> *ax, cx<T> *out) {
  if (DIM == 3) {
    cx<T> A[2][2];
    for (int by = 0; by < 2; ++by)
      for (int bz = 0; bz < 2; ++bz) {
        int b = 2 * by + 4 * bz;
        A[by][bz] = cadd(rmul(ax[0].fwd[0], v[b]), rmul(ax[0].fwd[1], v[b + 1]));
      }
    cx<T> B[2][2];
    for (int bz = 0; bz < 2; ++bz) {
      B[0][bz] = cadd(cmul(ax[1].fwd[0], A[0][bz]), cmul(ax[1].fwd[1], A[1][bz]));
      B[1][bz] = cadd(cmulc(ax[1].fwd[0], A[0][bz]), cmulc(ax[1].fwd[1], A[1][bz]));
    }
    for (int my = 0; my < 2; ++my) {
      out[my * 2 + 0] = cadd(cmul(ax[2].fwd[0], B[my][0]), cmul(ax[2].fwd[1], B[my][1]));
      out[my * 2 + 1] = cadd(cmulc(ax[2].fwd[0], B[my][0]), cmulc(ax[2].fwd[1], B[my][1]));
    }
  } else {
    cx<T> A[2];
    for (int by = 0; by < 2; ++by) A[by] = cadd(rmul(ax[0].fwd[0], v[2 * by]), rmul(ax[0].fwd[1], v[2 * by + 1]));
    out[0] = cadd(cmul(ax[1].fwd[0], A[0]), cmul(ax[1].fwd[1], A[1]));
    out[1] = cadd(cmulc(ax[1].fwd[0], A[0]), cmulc(ax[1].fwd[1], A[1]));
  }
}

// Back transform: real nodal vector = 2 Re(sum over mu_x = + modes).
template <typename T, int DIM>
TR_HD void modes_backward(const cx<T> *U, const AxisXf<T> *ax, T *v) {
  if (DIM == 3) {
    cx<T> E[2][2];  // [my][bz]
    for (int my = 0; my < 2; ++my)
      for (int bz = 0; bz < 2; ++bz) {
        cx<T> c = ax[2].bwd[bz];
        cx<T> cc{c.re, -c.im};
        E[my][bz] = cadd(cmul(c, U[my * 2 + 0]), cmul(cc, U[my * 2 + 1]));
      }
    for (int by = 0; by < 2; ++by) {
      cx<T> c = ax[1].bwd[by];
      cx<T> cc{c.re, -c.im};
      for (int bz = 0; bz < 2; ++bz) {
        cx<T> F = cadd(cmul(c, E[0][bz]), cmul(cc, E[1][bz]));
        for (int bx = 0; bx < 2; ++bx) {
          cx<T> x = ax[0].bwd[bx];
          v[bx + 2 * by + 4 * bz] = T(2) * (x.re * F.re - x.im * F.im);
        }
      }
    }
  } else {
    for (int by = 0; by < 2; ++by) {
      cx<T> c = ax[1].bwd[by];
      cx<T> cc{c.re, -c.im};
      cx<T> F = cadd(cmul(c, U[0]), cmul(cc, U[1]));
      for (int bx = 0; bx < 2; ++bx) {
        cx<T> x = ax[0].bwd[bx];
        v[bx + 2 * by] = T(2) * (x.re * F.re - x.im * F.im);
      }
    }
  }
}

// Mode eigenvalue D_mu = sigma + sum_xi c_xi lambda_{mu_xi}, lambda = 2 +- i sqrt 2.
template <typename T, int DIM>
TR_HD cx<T> mode_eig(int mode, const T *c, T sigma) {
  const T r2 = T(1.41421356237309504880);
  T re = sigma + T(2) * (c[0] + c[1] + (DIM == 3 ? c[2] : T(0)));
  T sy = (DIM == 3 ? (mode >> 1) : mode) ? T(-1) : T(1);
  T sz = (DIM == 3 && (mode & 1)) ? T(-1) : T(1);
  T im = r2 * (c[0] + sy * c[1] + (DIM == 3 ? sz * c[2] : T(0)));
  return {re, im};
}

// Solve (sum_xi c_xi E_xi + sigma I) u = v (or its transpose) in place.
template <typename T, int DIM, bool TRANS>
TR_HD void spectral_solve(T *v, const T *c, T sigma, int flip) {
  constexpr int NM = DIM == 3 ? 4 : 2;
  AxisXf<T> ax[3];
  for (int d = 0; d < DIM; ++d) ax[d] = axis_xf<T>((flip >> d) & 1, TRANS);
  cx<T> m[NM];
  modes_forward<T, DIM>(v, ax, m);
  for (int k = 0; k < NM; ++k) m[k] = cmul(m[k], cinv(mode_eig<T, DIM>(k, c, sigma)));
  modes_backward<T, DIM>(m, ax, v);
}

// Apply the cell mass matrix shape (N-hat = [[2,1],[1,2]]/6 per axis) or
// its inverse (2 [[2,-1],[-1,2]] per axis), without the cell volume.
template <typename T, int DIM, bool INV>
TR_HD void mass_shape(T *v) {
  constexpr int NS = 1 << DIM;
  for (int d = 0; d < DIM; ++d) {
    int bit = 1 << d;
    for (int b = 0; b < NS; ++b) {
      if (b & bit) continue;
      T a = v[b], e = v[b | bit];
      if (INV) {
        v[b] = T(4) * a - T(2) * e;
        v[b | bit] = T(4) * e - T(2) * a;
      } else {
        v[b] = (T(2) * a + e) * T(1.0 / 6.0);
        v[b | bit] = (a + T(2) * e) * T(1.0 / 6.0);
      }
    }
  }
}

// ------------------------------------------------------------------------
// Specialised form of spectral_solve for an orientation known at compile
// time.  The per-axis transforms are written out with their constant
// coefficients (no multiplications by 0 or 1), and each forward or back
// transform is taken without its factor q = 1/(2 sqrt 2) per axis; the
// missing q^DIM, the factor 2 of the real part and the eigenvalue division
// are applied together to each mode.  In oriented node order (x0 upstream,
// x1 downstream) with s2 = sqrt 2:
//   forward        m+- = s2 x0 -+ i (x0 + x1)            (times q)
//   back           x0 = U+ + U-,  x1 = -(U+ + U-) + i s2 (U+ - U-)
//   forward^T      m+- = (x0 - x1) +- i s2 x1
//   back^T         x0 = s2 (U+ + U-) - i (U+ - U-),  x1 = -i (U+ - U-)   (times q)
// On the first axis only the mu = + mode is formed (real input) and on the
// last back transform only the real part is taken.

// Per-ordinate constants of the mode eigenvalues D_k = sigma + c2 + i im[k].
template <typename T, int DIM>
struct ModeConst {
  T c2;         // 2 (c_x + c_y + c_z)
  T im[4];      // sqrt 2 (c_x +- c_y +- c_z), mode k = my * 2 + mz (3-D) or my (2-D)
  T im2[4];     // im[k]^2
};

template <typename T, int DIM>
TR_HD ModeConst<T, DIM> mode_const(const T *c) {
  const T r2 = T(1.41421356237309504880);
  ModeConst<T, DIM> m;
  m.c2 = T(2) * (c[0] + c[1] + (DIM == 3 ? c[2] : T(0)));
  for (int k = 0; k < (DIM == 3 ? 4 : 2); ++k) {
    T sy = (DIM == 3 ? (k >> 1) : k) ? T(-1) : T(1);
    T sz = (DIM == 3 && (k & 1)) ? T(-1) : T(1);
    m.im[k] = r2 * (c[0] + sy * c[1] + (DIM == 3 ? sz * c[2] : T(0)));
    m.im2[k] = m.im[k] * m.im[k];
  }
  return m;
}

// 1 / x for x > 0 in the normal range: hardware reciprocal estimate and two
// Newton steps (double) or the estimate alone (float, 1 ulp).
TR_HD double fast_rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
#else
  return 1.0 / x;
#endif
}
TR_HD float fast_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// forward pair, complex input (upstream x0, downstream x1) -> (m+, m-)
template <typename T, bool TRANS>
TR_HD void fwd_pair(cx<T> x0, cx<T> x1, cx<T> &mp, cx<T> &mm) {
  const T r2 = T(1.41421356237309504880);
  if (!TRANS) {
    const cx<T> s{x0.re + x1.re, x0.im + x1.im}, t{r2 * x0.re, r2 * x0.im};
    mp = {t.re + s.im, t.im - s.re};
    mm = {t.re - s.im, t.im + s.re};
  } else {
    const cx<T> d{x0.re - x1.re, x0.im - x1.im}, e{r2 * x1.re, r2 * x1.im};
    mp = {d.re - e.im, d.im + e.re};
    mm = {d.re + e.im, d.im - e.re};
  }
}

// back pair (U+, U-) -> complex node values (upstream x0, downstream x1)
template <typename T, bool TRANS>
TR_HD void bwd_pair(cx<T> up, cx<T> um, cx<T> &x0, cx<T> &x1) {
  const T r2 = T(1.41421356237309504880);
  const cx<T> P{up.re + um.re, up.im + um.im}, M{up.re - um.re, up.im - um.im};
  if (!TRANS) {
    x0 = P;
    x1 = {-P.re - r2 * M.im, -P.im + r2 * M.re};
  } else {
    x0 = {r2 * P.re + M.im, r2 * P.im - M.re};
    x1 = {M.im, -M.re};
  }
}

// Solve (sum_xi c_xi E_xi + sigma I) u = v (TRANS: the transpose) in place
// for the orientation FLIP; result identical to spectral_solve up to rounding.
template <typename T, int DIM, bool TRANS, int FLIP>
TR_HD void oriented_solve(T *v, const ModeConst<T, DIM> &mc, T sigma) {
  const T r2 = T(1.41421356237309504880);
  constexpr int fx = FLIP & 1, fy = (FLIP >> 1) & 1, fz = (FLIP >> 2) & 1;
  // q^DIM times the factor 2 of the real part
  const T kappa = DIM == 3 ? T(0.08838834764831844055) : T(0.25);
  if (DIM == 3) {
    cx<T> A[2][2];  // [by][bz], x-mode +
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bz = 0; bz < 2; ++bz) {
        const T x0 = v[fx + 2 * by + 4 * bz], x1 = v[(1 - fx) + 2 * by + 4 * bz];
        A[by][bz] = TRANS ? cx<T>{x0 - x1, r2 * x1} : cx<T>{r2 * x0, -(x0 + x1)};
      }
    cx<T> B[2][2];  // [my][bz]
#pragma unroll
    for (int bz = 0; bz < 2; ++bz) fwd_pair<T, TRANS>(A[fy][bz], A[1 - fy][bz], B[0][bz], B[1][bz]);
    cx<T> m[4];
#pragma unroll
    for (int my = 0; my < 2; ++my) fwd_pair<T, TRANS>(B[my][fz], B[my][1 - fz], m[2 * my], m[2 * my + 1]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T re = sigma + mc.c2;
      const T f = kappa * fast_rcp(__builtin_fma(re, re, mc.im2[k]));
      const T a = (m[k].re * re + m[k].im * mc.im[k]) * f;
      const T b = (m[k].im * re - m[k].re * mc.im[k]) * f;
      m[k] = {a, b};
    }
    cx<T> E[2][2];  // [my][bz]
#pragma unroll
    for (int my = 0; my < 2; ++my) bwd_pair<T, TRANS>(m[2 * my], m[2 * my + 1], E[my][fz], E[my][1 - fz]);
    cx<T> F[2][2];  // [by][bz]
#pragma unroll
    for (int bz = 0; bz < 2; ++bz) bwd_pair<T, TRANS>(E[0][bz], E[1][bz], F[fy][bz], F[1 - fy][bz]);
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bz = 0; bz < 2; ++bz) {
        const cx<T> f = F[by][bz];
        v[fx + 2 * by + 4 * bz] = TRANS ? r2 * f.re + f.im : f.re;
        v[(1 - fx) + 2 * by + 4 * bz] = TRANS ? f.im : -f.re - r2 * f.im;
      }
  } else {
    cx<T> A[2];  // [by]
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const T x0 = v[fx + 2 * by], x1 = v[(1 - fx) + 2 * by];
      A[by] = TRANS ? cx<T>{x0 - x1, r2 * x1} : cx<T>{r2 * x0, -(x0 + x1)};
    }
    cx<T> m[2];
    fwd_pair<T, TRANS>(A[fy], A[1 - fy], m[0], m[1]);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const T re = sigma + mc.c2;
      const T f = kappa * fast_rcp(__builtin_fma(re, re, mc.im2[k]));
      const T a = (m[k].re * re + m[k].im * mc.im[k]) * f;
      const T b = (m[k].im * re - m[k].re * mc.im[k]) * f;
      m[k] = {a, b};
    }
    cx<T> F[2];
    bwd_pair<T, TRANS>(m[0], m[1], F[fy], F[1 - fy]);
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const cx<T> f = F[by];
      v[fx + 2 * by] = TRANS ? r2 * f.re + f.im : f.re;
      v[(1 - fx) + 2 * by] = TRANS ? f.im : -f.re - r2 * f.im;
    }
  }
}

}  // namespace tr
