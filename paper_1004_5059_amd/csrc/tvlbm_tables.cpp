// tvlbm_tables.cpp -- Gauss-Hermite velocity sets and host constants.
//
// Nodes: the roots of the probabilists' Hermite polynomial He_n, located by
// scanning for sign changes, bisected, then refined by Newton's method
// (He_n' = n He_{n-1}).  Weights: w_i = n! / (n^2 He_{n-1}(x_i)^2), the
// Gauss-Hermite weight for the normalised Gaussian measure.
#include "tvlbm_tables.h"

#include <cmath>
#include <cstring>

namespace tvlbm {

static void he_pair(int n, double x, double* hn, double* hnm1) {
  double a = 1.0, b = x;
  if (n == 0) { *hn = 1.0; *hnm1 = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    const double c = x * b - k * a;
    a = b;
    b = c;
  }
  *hn = b;
  *hnm1 = a;
}

bool gauss_hermite_rule(int n, double* x, double* w) {
  if (n < 2 || n > 8) return false;
  const double lim = std::sqrt(4.0 * n + 2.0) + 1.0;
  const int steps = 20000;
  int found = 0;
  double prev_x = -lim, prev_h, tmp;
  he_pair(n, prev_x, &prev_h, &tmp);
  for (int s = 1; s <= steps && found < n; ++s) {
    const double cx = -lim + 2.0 * lim * s / steps;
    double ch;
    he_pair(n, cx, &ch, &tmp);
    if (ch == 0.0) {
      x[found++] = cx;  // a root on the scan grid (x = 0 for odd n)
    } else if (prev_h != 0.0 && (ch < 0.0) != (prev_h < 0.0)) {
      double lo = prev_x, hi = cx, hlo = prev_h;
      for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        double hm;
        he_pair(n, mid, &hm, &tmp);
        if ((hm < 0.0) == (hlo < 0.0)) { lo = mid; hlo = hm; } else { hi = mid; }
      }
      double r = 0.5 * (lo + hi);
      for (int it = 0; it < 4; ++it) {
        double hn, hm1;
        he_pair(n, r, &hn, &hm1);
        if (hm1 != 0.0) r -= hn / (n * hm1);
      }
      x[found++] = r;
    }
    prev_x = cx;
    prev_h = ch;
  }
  if (found != n) return false;
  double fact = 1.0;
  for (int k = 2; k <= n; ++k) fact *= k;
  for (int i = 0; i < n; ++i) {
    double hn, hm1;
    he_pair(n, x[i], &hn, &hm1);
    w[i] = fact / (double(n) * n * hm1 * hm1);
  }
  // exact symmetry about the origin
  for (int i = 0; i < n / 2; ++i) {
    const double xa = 0.5 * (x[n - 1 - i] - x[i]), wa = 0.5 * (w[i] + w[n - 1 - i]);
    x[i] = -xa; x[n - 1 - i] = xa; w[i] = wa; w[n - 1 - i] = wa;
  }
  if (n % 2) x[n / 2] = 0.0;
  return true;
}

bool build_lattice(int n, int order, double cfl, int cfl_norm, HostLattice* L) {
  // order 5 (the 6-point rule integrates H5 H5 exactly) is for the
  // finite-volume path only; the lattice entry points reject it
  if (!((n == 3 && order == 2) || (n == 4 && order == 3) || (n == 6 && (order == 4 || order == 5))))
    return false;
  if (!(cfl > 0.0)) return false;
  *L = HostLattice();
  L->n = n;
  L->q = n * n;
  L->order = order;
  if (!gauss_hermite_rule(n, L->x, L->wx)) return false;
  const double xmax = L->x[n - 1];
  L->lambda = cfl / (cfl_norm == 0 ? std::sqrt(2.0) * xmax : xmax);
  for (int a = 0; a < n; ++a) {
    double s = std::fabs(L->lambda * L->x[a]);
    const double r = std::nearbyint(s);
    if (std::fabs(s - r) <= 4.0 * (std::nextafter(s, 2.0 * s + 1.0) - s)) s = r;
    if (s > 1.0) return false;
    L->p[a] = s;
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const int l = a * n + b;
      L->xi[2 * l] = L->x[a];
      L->xi[2 * l + 1] = L->x[b];
      L->w[l] = L->wx[a] * L->wx[b];
      L->shift[2 * l] = (L->x[a] < 0 ? -1.0 : 1.0) * L->p[a];
      L->shift[2 * l + 1] = (L->x[b] < 0 ? -1.0 : 1.0) * L->p[b];
    }
  return true;
}

void host_feq(const HostLattice& L, double rho, double ux, double uy, double T, double* feq) {
  const double D = 2.0, u2 = ux * ux + uy * uy, th = T - 1.0;
  for (int l = 0; l < L.q; ++l) {
    const double cx = L.xi[2 * l], cy = L.xi[2 * l + 1];
    const double ul = ux * cx + uy * cy, c2 = cx * cx + cy * cy, ul2 = ul * ul;
    double P = 1.0 + ul + 0.5 * (ul2 - u2 + th * (c2 - D));
    if (L.order >= 3) P += ul / 6.0 * (ul2 - 3.0 * u2 + 3.0 * th * (c2 - D - 2.0));
    if (L.order >= 4)
      P += (ul2 * ul2 - 6.0 * ul2 * u2 + 3.0 * u2 * u2) / 24.0 +
           th / 4.0 * ((c2 - D - 2.0) * (ul2 - u2) - 2.0 * ul2) +
           th * th / 8.0 * (c2 * c2 - 2.0 * (D + 2.0) * c2 + D * (D + 2.0));
    if (L.order >= 5) {
      const double ul3 = ul2 * ul;
      P += (ul3 * ul2 - 10.0 * u2 * ul3 + 15.0 * u2 * u2 * ul) / 120.0 +
           th / 12.0 * (c2 * ul3 - (D + 6.0) * ul3 - 3.0 * c2 * ul * u2 + (3.0 * D + 12.0) * u2 * ul) +
           th * th / 8.0 * (ul * c2 * c2 - (2.0 * D + 8.0) * c2 * ul + (D * D + 6.0 * D + 8.0) * ul);
    }
    feq[l] = L.w[l] * rho * P;
  }
}

}  // namespace tvlbm
