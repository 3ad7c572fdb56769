// tvlbm_tables.h -- host-side lattice tables of the library (Gauss-Hermite
// rule, displacements, equilibrium in double precision for wall constants).
#pragma once

#include <stdint.h>

namespace tvlbm {

struct HostLattice {
  int n = 0, q = 0, order = 0;
  double x[8] = {0}, wx[8] = {0};   // 1-D rule, ascending nodes
  double p[8] = {0};                // |displacement| per node, snapped
  double lambda = 0.0;
  double xi[2 * 36] = {0}, w[36] = {0}, shift[2 * 36] = {0};
};

// 1-D Gauss-Hermite rule (probabilists' weight, sum 1) for n points.
// Returns false on bad n.
bool gauss_hermite_rule(int n, double* x, double* w);

// Builds the tensor-product lattice; false if n/order unsupported or a
// displacement exceeds one cell.
bool build_lattice(int n, int order, double cfl, int cfl_norm, HostLattice* L);

// Hermite equilibrium (double) of the lattice at (rho, ux, uy, T).
void host_feq(const HostLattice& L, double rho, double ux, double uy, double T, double* feq);

}  // namespace tvlbm
