// Host build of the library's angular setup (angular_setup.cpp) for the CPU
// tests, compiled with the address and undefined-behaviour sanitizers: it
// builds the patch tree and levels for a refinement spec, forms the finest
// level's scatter matrix for HG moments, and writes every table as raw
// doubles (each array preceded by its length as a double).
//   setup_dump base cone_x cone_y cone_z half_angle extra closure band_lmax order g basis out.bin
// (basis 0 = Lin, 1 = Const)
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2010_04559_amd/csrc/angular_setup.h"

static void put(FILE *f, const std::vector<double> &v) {
  const double n = (double)v.size();
  std::fwrite(&n, sizeof n, 1, f);
  if (!v.empty()) std::fwrite(v.data(), sizeof(double), v.size(), f);
}

int main(int argc, char **argv) {
  if (argc != 13) {
    std::fprintf(stderr, "usage: setup_dump base cx cy cz half extra closure band order g basis out\n");
    return 2;
  }
  tr::RefineSpec spec;
  spec.base_level = std::atoi(argv[1]);
  spec.cone_axis = {std::atof(argv[2]), std::atof(argv[3]), std::atof(argv[4])};
  spec.cone_half_angle_deg = std::atof(argv[5]);
  spec.cone_extra_levels = std::atoi(argv[6]);
  spec.closure = std::atoi(argv[7]) != 0;
  spec.band_lmax = std::atoi(argv[8]);
  const int order = std::atoi(argv[9]);
  const double g = std::atof(argv[10]);
  spec.const_basis = std::atoi(argv[11]) != 0;
  tr::HostAngular ang;
  std::string err;
  if (!tr::build_angular(spec, ang, err)) {
    std::fprintf(stderr, "build_angular: %s\n", err.c_str());
    return 1;
  }
  FILE *f = std::fopen(argv[12], "wb");
  if (!f) return 1;
  put(f, {(double)ang.lv.size()});
  for (const tr::HostLevel &L : ang.lv) {
    put(f, {(double)L.P});
    std::vector<double> verts;
    for (int q = 0; q < L.P; ++q) {
      const tr::PatchNode &p = ang.tree[L.node[q]];
      for (int v = 0; v < 3; ++v) {
        verts.push_back(p.v[v].x);
        verts.push_back(p.v[v].y);
        verts.push_back(p.v[v].z);
      }
    }
    put(f, verts);
    put(f, L.omega);
    put(f, L.w);
    put(f, L.ipsi);
    put(f, L.iom);
    put(f, std::vector<double>(L.owner.begin(), L.owner.end()));
    put(f, L.pblk);
  }
  std::vector<double> mom(order + 1), St;
  double gn = 1.0;
  for (int n = 0; n <= order; ++n, gn *= g) mom[n] = gn;
  tr::scatter_matrix(ang, (int)ang.lv.size() - 1, mom, St);
  put(f, St);
  std::fclose(f);
  return 0;
}
