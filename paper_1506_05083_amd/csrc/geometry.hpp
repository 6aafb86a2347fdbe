// Host-side geometry helpers (see geometry.cpp).
#pragma once

#include <complex>
#include <vector>

#include "../../include/mfs.h"

namespace mfs {

struct RBOrder {
  int m, n;
  double kx, ky;
  std::complex<double> kz;
};

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
void polar_geometry(const mfs_polar_spec &s, double *rho, double *z, double *nrho, double *nz,
                    double *srho, double *sz);
void cup_geometry(const mfs_cup_spec &s, double *rho, double *z, double *nrho, double *nz, double *srho,
                  double *sz);
// SoA [6 walls R L F B T D][x y z][M1^2]
void wall_nodes(const mfs_lattice &lat, std::vector<double> &soa);
void rb_orders(double k, const double kv[3], const mfs_lattice &lat, std::vector<RBOrder> &out);

}  // namespace mfs
