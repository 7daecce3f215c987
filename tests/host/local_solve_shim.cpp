// Host build of the library's per-cell ordinate solve (local_solve.h) for
// the CPU tests: the forward solve (sum_xi c_xi E_xi + sigma I)^{-1} v and
// the transposed one followed by the inverse cell mass shape, for every
// orientation, exported with C linkage.
#include "../../paper_2010_04559_amd/csrc/local_solve.h"

namespace {
template <int DIM, bool TRANS, int FLIP>
void run(double *v, const double *c, double sigma) {
  const tr::ModeConst<double, DIM> mc = tr::mode_const<double, DIM>(c);
  tr::oriented_solve<double, DIM, TRANS, FLIP>(v, mc, sigma);
  if (TRANS) tr::mass_shape<double, DIM, true>(v);
}
template <int DIM, bool TRANS>
void dispatch(int flip, double *v, const double *c, double sigma) {
  switch (flip) {
    case 0: run<DIM, TRANS, 0>(v, c, sigma); break;
    case 1: run<DIM, TRANS, 1>(v, c, sigma); break;
    case 2: run<DIM, TRANS, 2>(v, c, sigma); break;
    case 3: run<DIM, TRANS, 3>(v, c, sigma); break;
    case 4: run<DIM, TRANS, 4>(v, c, sigma); break;
    case 5: run<DIM, TRANS, 5>(v, c, sigma); break;
    case 6: run<DIM, TRANS, 6>(v, c, sigma); break;
    default: run<DIM, TRANS, 7>(v, c, sigma); break;
  }
}
}  // namespace

extern "C" void ls_solve(int dim, int trans, int flip, double *v, const double *c, double sigma) {
  if (dim == 3)
    trans ? dispatch<3, true>(flip, v, c, sigma) : dispatch<3, false>(flip, v, c, sigma);
  else
    trans ? dispatch<2, true>(flip & 3, v, c, sigma) : dispatch<2, false>(flip & 3, v, c, sigma);
}

// the spectral form for a run-time orientation (the register sweep's solve),
// with the same inverse mass shape after the transposed solve
extern "C" void ls_spectral(int dim, int trans, int flip, double *v, const double *c, double sigma) {
  if (dim == 3) {
    if (trans) {
      tr::spectral_solve<double, 3, true>(v, c, sigma, flip);
      tr::mass_shape<double, 3, true>(v);
    } else {
      tr::spectral_solve<double, 3, false>(v, c, sigma, flip);
    }
  } else {
    if (trans) {
      tr::spectral_solve<double, 2, true>(v, c, sigma, flip & 3);
      tr::mass_shape<double, 2, true>(v);
    } else {
      tr::spectral_solve<double, 2, false>(v, c, sigma, flip & 3);
    }
  }
}
