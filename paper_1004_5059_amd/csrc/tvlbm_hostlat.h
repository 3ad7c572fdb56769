// tvlbm_hostlat.h -- the lattice constants of the device parameter block
// (Lat<R>) from the host tables.
#pragma once

#include <cmath>
#include <cstring>
#include <type_traits>

#include "tvlbm_core.h"
#include "tvlbm_tables.h"

namespace tvlbm {

template <typename R>
inline void fill_lat(const HostLattice& H, Lat<R>& L) {
  std::memset(&L, 0, sizeof L);
  const int n = H.n;
  for (int a = 0; a < n; ++a) {
    // round the pull fraction to the dtype's unit-interval grid so that
    // (1 - p) + p == 1 exactly in that dtype
    const double ulp = std::is_same<R, float>::value ? 0x1p-24 : 0x1p-53;
    const double p = std::nearbyint(H.p[a] / ulp) * ulp;
    L.p[a] = (R)p;
    L.qm[a] = (R)(1.0 - p);
    L.x[a] = (R)H.x[a];
    L.x2[a] = (R)(H.x[a] * H.x[a]);
    L.xd[a] = H.x[a];
  }
  double sw = 0.0;
  for (int l = 0; l < H.q; ++l) {
    L.w[l] = (R)H.w[l];
    L.wd[l] = H.w[l];
    sw += H.w[l];
  }
  L.sumw = sw;
}

}  // namespace tvlbm
