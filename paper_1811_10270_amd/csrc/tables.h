// Host-side construction of the constant tables the kernels read: Gauss-
// Legendre rules, normalised associated Legendre values and theta
// derivatives at grid latitudes, longitude trigonometric tables, modified
// singular weights, and the real rotation matrices built from Wigner small-d.
#pragma once
#include <vector>

#if defined(__HIPCC__)
#define EHD_HD __host__ __device__
#else
#define EHD_HD
#endif

namespace ehd {

EHD_HD inline long ncoef(int p) { return (long)(p + 1) * (p + 2) / 2; }
EHD_HD inline long tri(int n, int m) { return (long)n * (n + 1) / 2 + m; }
EHD_HD inline int nlon_of(int P, int grid_mode) { return grid_mode == 0 ? 2 * P + 2 : 2 * P; }
// doubles in one rotation table block (all n <= p): sum_n (n+1)^2
EHD_HD inline long wig_block(int p) { return (long)(p + 1) * (p + 2) * (2 * p + 3) / 6; }
EHD_HD inline long wig_off(int n) { return (long)n * (n + 1) * (2 * n + 1) / 6; }

// Gauss-Legendre nodes (cos theta, theta increasing) and weights, n points.
void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w);

// Pbar_n^m(cos theta_i) and dPbar_n^m/dtheta at each latitude of a grid,
// [i][tri(n,m)], n <= p.
void legendre_tables(int p, const std::vector<double>& t, std::vector<double>& P,
                     std::vector<double>& dP);

// Wigner small-d matrix, d[(m+n)*(2n+1) + (m'+n)] = d^n_{m m'}(beta), with
// Y_nm(Ry(beta) v) = sum_m' d^n_{m m'}(beta) Y_nm'(v).
void wigner_d(int n, double beta, std::vector<double>& d);

// Real rotation blocks for one polar angle beta, n = 0..p:
//   A[wig_off(n) + m*(n+1) + m'] = d_{m m'} + (-1)^m d_{-m, m'}   (m >= 1)
//                                 = d_{0 m'}                      (m = 0)
//   B[...]                       = d_{m m'} - (-1)^m d_{-m, m'}   (m >= 1), 0 (m = 0)
// so that for z_m = c_nm e^{i m phi}:  Re c'_{nm'} = sum_m A Re z_m,
// Im c'_{nm'} = sum_m B Im z_m.
void rotation_blocks(int p, double beta, double* A, double* B);

// Modified weight factor of the singular rule on the degree-Q grid:
// msum_i = 2 sin(theta_i / 2) * sum_{n=0}^{Q} P_n(cos theta_i).
void singular_factor(int Q, const std::vector<double>& t, std::vector<double>& msum);

}  // namespace ehd
