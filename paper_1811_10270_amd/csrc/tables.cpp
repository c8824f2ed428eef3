// Constant tables for the kernels (host FP64).  See tables.h.
//
// Definitions: Gaussian grid and normalised SH with Condon-Shortley phase
// (paper Sec. 2, eq. normalized_spharm, eq. pneg); modified weights (Sec. 2.1,
// eq. mod_weights, with the Legendre sum taken to the degree of the grid the
// rule is applied on); the rotation that brings a target to the pole.
#include "tables.h"

#include <cmath>
#include <stdexcept>

namespace ehd {

static const double kPi = 3.14159265358979323846;

void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w)
{
    t.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        // Tricomi-type first guess, then Newton on P_n with the derivative
        // from (1 - x^2) P_n' = n (P_{n-1} - x P_n).
        double x = std::cos(kPi * (4.0 * i + 3.0) / (4.0 * n + 2.0)) *
                   (1.0 - (n - 1.0) / (8.0 * n * n * n));
        double dpn = 1.0;
        int fine = 0;   // Newton steps taken once |dx| <= 1e-12: the error after one is about n^2 dx^2
        for (int it = 0; it < 64 && fine < 2; ++it) {
            double a = 1.0, b = x;  // P_0, P_1
            if (n == 1) { a = 1.0; b = x; }
            for (int k = 1; k < n; ++k) {
                double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
                a = b;
                b = c;
            }
            double pn = (n == 0) ? 1.0 : b, pnm1 = a;
            dpn = n * (pnm1 - x * pn) / (1.0 - x * x);
            double dx = pn / dpn;
            x -= dx;
            if (std::fabs(dx) <= 1e-12 * (1.0 + std::fabs(x))) ++fine;
        }
        double a = 1.0, b = x;
        for (int k = 1; k < n; ++k) {
            double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
            a = b;
            b = c;
        }
        dpn = n * (a - x * b) / (1.0 - x * x);
        t[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dpn * dpn);
    }
}

void legendre_tables(int p, const std::vector<double>& t, std::vector<double>& P,
                     std::vector<double>& dP)
{
    const int nlat = (int)t.size();
    const long nc = ncoef(p);
    P.assign((size_t)nlat * nc, 0.0);
    dP.assign((size_t)nlat * nc, 0.0);
    // values up to degree p+1 in m (needed by the ladder formula for m+1);
    // the square-root factors do not depend on the point
    const int pp = p + 1;
    std::vector<double> row(ncoef(pp)), fd(pp + 1), fs(pp + 1), fa(ncoef(pp)), fb(ncoef(pp)), fu(nc), fn(nc);
    for (int m = 0; m <= pp; ++m) {
        fd[m] = m > 0 ? std::sqrt((2.0 * m + 1.0) / (2.0 * m)) : 0.0;
        fs[m] = std::sqrt(2.0 * m + 3.0);
        for (int n = m + 2; n <= pp; ++n) {
            fa[tri(n, m)] = std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
            fb[tri(n, m)] = std::sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
        }
    }
    // ladder: dP/dtheta = 1/2 [ sqrt((n-m)(n+m+1)) P^{m+1} - sqrt((n+m)(n-m+1)) P^{m-1} ],
    // with P_n^{-1} = -P_n^1.
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
            fu[tri(n, m)] = (m + 1 <= n) ? std::sqrt((double)(n - m) * (n + m + 1)) : 0.0;
            fn[tri(n, m)] = m >= 1 ? std::sqrt((double)(n + m) * (n - m + 1)) : (n >= 1 ? -std::sqrt((double)n * (n + 1)) : 0.0);
        }
    for (int i = 0; i < nlat; ++i) {
        const double x = t[i], s = std::sqrt((1.0 - x) * (1.0 + x));
        double diag = 1.0 / std::sqrt(4.0 * kPi);
        for (int m = 0; m <= pp; ++m) {
            if (m > 0) diag *= -fd[m] * s;
            row[tri(m, m)] = diag;
            if (m + 1 <= pp) row[tri(m + 1, m)] = fs[m] * x * diag;
            for (int n = m + 2; n <= pp; ++n)
                row[tri(n, m)] = fa[tri(n, m)] * (x * row[tri(n - 1, m)] - fb[tri(n, m)] * row[tri(n - 2, m)]);
        }
        for (int n = 0; n <= p; ++n) {
            for (int m = 0; m <= n; ++m) {
                const long k = tri(n, m);
                P[(size_t)i * nc + k] = row[k];
                const double up = (m + 1 <= n) ? fu[k] * row[tri(n, m + 1)] : 0.0;
                const double dn = m >= 1 ? fn[k] * row[tri(n, m - 1)] : (n >= 1 ? fn[k] * row[tri(n, 1)] : 0.0);
                dP[(size_t)i * nc + k] = 0.5 * (up - dn);
            }
        }
    }
}

// log of n! via lgamma is accurate enough for the seed coefficients; the
// binomial is formed as exp of a difference to avoid overflow.
static double sqrt_binom(int a, int b)  // sqrt(a! / (b! (a-b)!))
{
    return std::exp(0.5 * (std::lgamma(a + 1.0) - std::lgamma(b + 1.0) - std::lgamma(a - b + 1.0)));
}

void wigner_d(int n, double beta, std::vector<double>& d)
{
    const int N = 2 * n + 1;
    d.assign((size_t)N * N, 0.0);
    const double cb = std::cos(beta), ch = std::cos(0.5 * beta), sh = std::sin(0.5 * beta);
    for (int m = -n; m <= n; ++m) {
        for (int mp = -n; mp <= n; ++mp) {
            const int j0 = std::max(std::abs(m), std::abs(mp));
            // seed d^{j0}_{m mp}
            double seed;
            if (j0 == std::abs(m) && (std::abs(m) >= std::abs(mp))) {
                const int j = j0, b = mp;
                if (m >= 0)
                    seed = (((j - b) & 1) ? -1.0 : 1.0) * sqrt_binom(2 * j, j + b) *
                           std::pow(ch, j + b) * std::pow(sh, j - b);
                else
                    seed = sqrt_binom(2 * j, j + b) * std::pow(ch, j - b) * std::pow(sh, j + b);
            } else {
                // |mp| > |m|: d^j_{m, mp} = (-1)^{m - mp} d^j_{mp, m}
                const int j = j0, b = m;
                double t;
                if (mp >= 0)
                    t = (((j - b) & 1) ? -1.0 : 1.0) * sqrt_binom(2 * j, j + b) *
                        std::pow(ch, j + b) * std::pow(sh, j - b);
                else
                    t = sqrt_binom(2 * j, j + b) * std::pow(ch, j - b) * std::pow(sh, j + b);
                seed = (((m - mp) & 1) ? -1.0 : 1.0) * t;
            }
            if (j0 > n) continue;
            double dm2 = 0.0, dm1 = seed;
            double val = (j0 == n) ? seed : 0.0;
            if (j0 == 0) {
                // m = mp = 0: Legendre polynomials P_j(cos beta)
                double a = 1.0, b = cb;
                if (n == 0) val = 1.0;
                else {
                    for (int j = 1; j < n; ++j) {
                        double c = ((2.0 * j + 1.0) * cb * b - j * a) / (j + 1.0);
                        a = b;
                        b = c;
                    }
                    val = b;
                }
            } else {
                for (int j = j0 + 1; j <= n; ++j) {
                    const double mm = (double)m * m, pp = (double)mp * mp;
                    const double c1 = (2.0 * j - 1.0) * (j * (j - 1.0) * cb - (double)m * mp);
                    const double c2 = j * std::sqrt(((j - 1.0) * (j - 1.0) - mm) * ((j - 1.0) * (j - 1.0) - pp));
                    const double c0 = (j - 1.0) * std::sqrt(((double)j * j - mm) * ((double)j * j - pp));
                    const double dj = (c1 * dm1 - c2 * dm2) / c0;
                    dm2 = dm1;
                    dm1 = dj;
                }
                val = dm1;
            }
            d[(size_t)(m + n) * N + (mp + n)] = val;
        }
    }
}

void rotation_blocks(int p, double beta, double* A, double* B)
{
    std::vector<double> d;
    for (int n = 0; n <= p; ++n) {
        wigner_d(n, beta, d);
        const int N = 2 * n + 1;
        double* An = A + wig_off(n);
        double* Bn = B + wig_off(n);
        for (int m = 0; m <= n; ++m) {
            for (int mp = 0; mp <= n; ++mp) {
                const double dpos = d[(size_t)(m + n) * N + (mp + n)];
                if (m == 0) {
                    An[m * (n + 1) + mp] = dpos;
                    Bn[m * (n + 1) + mp] = 0.0;
                } else {
                    const double sgn = (m & 1) ? -1.0 : 1.0;
                    const double dneg = d[(size_t)(-m + n) * N + (mp + n)];
                    An[m * (n + 1) + mp] = dpos + sgn * dneg;
                    Bn[m * (n + 1) + mp] = dpos - sgn * dneg;
                }
            }
        }
    }
}

void singular_factor(int Q, const std::vector<double>& t, std::vector<double>& msum)
{
    msum.assign(t.size(), 0.0);
    for (size_t i = 0; i < t.size(); ++i) {
        const double x = t[i];
        double a = 1.0, b = x, acc = 1.0 + (Q >= 1 ? x : 0.0);
        for (int k = 1; k < Q; ++k) {
            double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
            a = b;
            b = c;
            acc += c;
        }
        msum[i] = std::sqrt(2.0 * (1.0 - x)) * acc;
    }
}

}  // namespace ehd
