// Host-side angular discretisation for the HIP transport library.
//
// Builds the hierarchical octahedral patch tree (Section 2.1), the nested
// meshes T_l (Section 4.1), the Lin basis (Section 2.2), the collocated
// 3-point rule of the transport terms, the X integrals of eq. X with the
// dense scatter matrices S~ (Section 5.2), and the prolongation blocks
// (Section 4.1).  Plain C++, no device code.
#pragma once

#include <string>
#include <vector>

namespace tr {

struct V3 {
  double x, y, z;
};

struct PatchNode {
  V3 v[3];
  int level = 0, octant = 0, parent = -1;
  int child[4] = {-1, -1, -1, -1};
  bool leaf() const { return child[0] < 0; }
};

struct RefineSpec {
  int base_level = 0;
  V3 cone_axis{1, 0, 0};
  double cone_half_angle_deg = 0;
  int cone_extra_levels = 0;
  bool closure = true;
  // Section 5.5's z-band rule instead of the uniform level (0 = off): level
  // band_lmax where the largest vertex Omega_z exceeds 0.97, one less above
  // 0.9, two less above 0.8, three less above 0.6, four less elsewhere
  // (at least 0)
  int band_lmax = 0;
  // the Const basis of Section 2.2 carried as three coincident ordinates
  // per patch (mean direction, a third of the area each; see tr.h)
  bool const_basis = false;
};

// One nested angular mesh T_l with everything the kernels need.
struct HostLevel {
  int P = 0, A = 0;                 // patches, angular dofs (= ordinates)
  std::vector<int> node;            // tree node of each patch
  std::vector<int> octant;          // [P]
  std::vector<double> omega;        // [A][3] ordinate directions (3-point rule)
  std::vector<double> w;            // [A] weights (integrate psi_m exactly)
  std::vector<double> ipsi;         // [A] int psi_m
  std::vector<double> iom;          // [A][3] int Omega^xi psi_m (3-point rule)
  // prolongation from T_{l-1} (level l >= 1): owner patch on T_{l-1} and the
  // 3x3 block Pblk[c][k][d] = psi_{owner,d}(vertex k of c)
  std::vector<int> owner;           // [P]
  std::vector<double> pblk;         // [P][3][3]
  std::vector<int> first_child, n_child;  // [P_{l-1}] children on this level
};

struct HostAngular {
  std::vector<PatchNode> tree;
  std::vector<HostLevel> lv;        // T_0 .. T_L
  bool const_basis = false;
};

// Build the tree and levels.  Returns false with a message on bad input.
bool build_angular(const RefineSpec &spec, HostAngular &out, std::string &err);

// Dense canonical scatter matrix S~ = X F X^T (A x A, row-major) of a level
// for moments f_0..f_L (sigma_{s,n} = sigma_s f_n), from accurately
// integrated X integrals (eq. X); Xout (optional) receives X (A x K,
// K = (L+1)^2, harmonic index n^2 + n + o).
void scatter_matrix(const HostAngular &ang, int level, const std::vector<double> &moments,
                    std::vector<double> &St, std::vector<double> *Xout = nullptr);

// Accurate integral of psi_m * Y_{n,o} over a patch for n <= order; used
// for the X integrals.  X is [3][(order+1)^2].  With const_basis every row
// is a third of int_q Y_{n,o} (the Const function split over the three
// coincident ordinates).
void patch_x_integrals(const PatchNode &p, int order, std::vector<double> &X, bool const_basis = false);

// Lin basis values psi_d(omega) of a patch (barycentric coordinates of the
// gnomonic projection).
void lin_basis(const PatchNode &p, const V3 &om, double psi[3]);

double spherical_area(const PatchNode &p);

}  // namespace tr
