/*
 * ehd_oracle.c -- plain, slow, FP64 CPU oracle for the layer-potential
 * evaluation of Sorgentone, Tornberg & Vlahovska (arXiv 1811.10270).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP path.
 *
 * Route: every spherical-harmonic (SH) expansion is evaluated directly at the
 * physical points the quadrature needs.  The singular self-interaction rotates
 * the *points* (target to the north pole of a rotated Gaussian grid) and
 * evaluates the unrotated expansion there; no rotated coefficients, Wigner
 * matrices, GEMMs or FFTs are used.
 *
 * Definitions followed (paper sections / equations):
 *   Gaussian grid ............ Sec. 2, text after eq. spharm_ex
 *   normalised SH, CS phase .. Sec. 2, eq. normalized_spharm, eq. pneg
 *   regular quadrature ....... Sec. 2.1, eq. reg_quadrature
 *   modified (singular) weights Sec. 2.1, eq. mod_weights, and the rotation
 *                              of the target to the pole described after it
 *   Stokeslet / stresslet .... Sec. 1, eq. GandT
 *   S, D operators ........... Sec. 2, eq. op_stokes
 *   Laplace double layer L ... Sec. 2, eq. dl_op_laplace
 *   adjoint double layer K* .. the kernel of eq. E_n (normal at the target)
 *   Laplace single layer S_L . (1/4pi) int sigma/r dS (same prefactor as the
 *                              other operators; the paper uses its gradient
 *                              in eq. BIE01)
 *
 * Readings where the paper is ambiguous (each listed in the design notes):
 *   grid_mode 0: 2P+2 longitudes, weight 2pi/(2P+2); grid_mode 1: 2P
 *   longitudes, weight 2pi/(2P).  Modified-weight Legendre sum runs to the
 *   degree Q of the grid it is applied on.  Rotation R = Rz(phi_t) Ry(theta_t),
 *   third Euler angle 0.  The far sum excludes the target's own drop.
 *
 * Output components, in this order: S_x S_y S_z D_x D_y D_z S_L L K*.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PI 3.14159265358979323846
#define NCOMP 9

static int nlon_of(int P, int grid_mode) { return grid_mode == 0 ? 2 * P + 2 : 2 * P; }
static long ncoef_of(int p) { return (long)(p + 1) * (p + 2) / 2; }
static long tri(int n, int m) { return (long)n * (n + 1) / 2 + m; }

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes by Newton's method on P_n; nodes ordered t descending
 * (theta ascending).                                                        */
int ora_gauss_legendre(int n, double* t, double* w)
{
    if (n < 1) return 1;
    for (int i = 0; i < n; ++i) {
        double z = cos(ORA_PI * (i + 0.75) / (n + 0.5));
        double pp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pk = z, pkm1 = 1.0;
            for (int k = 2; k <= n; ++k) {
                double pkp1 = ((2.0 * k - 1.0) * z * pk - (k - 1.0) * pkm1) / k;
                pkm1 = pk;
                pk = pkp1;
            }
            /* P_n = pk, P_{n-1} = pkm1 (for n == 1: pk = z, pkm1 = 1) */
            pp = n * (z * pk - pkm1) / (z * z - 1.0);
            double dz = pk / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* final derivative at the converged node */
        {
            double pk = z, pkm1 = 1.0;
            for (int k = 2; k <= n; ++k) {
                double pkp1 = ((2.0 * k - 1.0) * z * pk - (k - 1.0) * pkm1) / k;
                pkm1 = pk;
                pk = pkp1;
            }
            pp = n * (z * pk - pkm1) / (z * z - 1.0);
        }
        t[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Normalised associated Legendre functions written as
 *     Pbar_n^m(t) = s^m Q_n^m(t),  s = sin(theta), t = cos(theta),
 * with Q_n^m a polynomial in t.  Q obeys the usual three-term recurrence in
 * n; its t-derivative is obtained by differentiating that recurrence.  Then
 *     dPbar_n^m/dtheta = s^(m-1) (m t Q - s^2 dQ/dt)      (m >= 1)
 *                      = -s dQ/dt                          (m = 0)
 *     Pbar_n^m / s     = s^(m-1) Q                         (m >= 1)
 * which are regular at the poles.                                           */
static void leg_eval(int p, double t, double* Q, double* dQ)
{
    double qmm = 1.0 / sqrt(4.0 * ORA_PI);
    for (int m = 0; m <= p; ++m) {
        if (m > 0) qmm *= -sqrt((2.0 * m + 1.0) / (2.0 * m));
        Q[tri(m, m)] = qmm;
        dQ[tri(m, m)] = 0.0;
        if (m + 1 <= p) {
            double c = sqrt(2.0 * m + 3.0);
            Q[tri(m + 1, m)] = c * t * qmm;
            dQ[tri(m + 1, m)] = c * qmm;
        }
        for (int n = m + 2; n <= p; ++n) {
            double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
            double b = sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
            Q[tri(n, m)] = a * (t * Q[tri(n - 1, m)] - b * Q[tri(n - 2, m)]);
            dQ[tri(n, m)] = a * (Q[tri(n - 1, m)] + t * dQ[tri(n - 1, m)] - b * dQ[tri(n - 2, m)]);
        }
    }
}

/* Pbar_n^m(t) for all n,m <= p at one point (used by the pins and analysis). */
void ora_pbar(int p, double t, double s, double* out /* [tri] */,
              double* dtheta /* [tri] or NULL */, double* over_s /* [tri] or NULL */)
{
    long nc = ncoef_of(p);
    double* Q = (double*)malloc(sizeof(double) * nc);
    double* dQ = (double*)malloc(sizeof(double) * nc);
    leg_eval(p, t, Q, dQ);
    double sm = 1.0, smm1 = 0.0; /* s^m, s^(m-1) */
    for (int m = 0; m <= p; ++m) {
        if (m == 1) { smm1 = 1.0; sm = s; }
        else if (m > 1) { smm1 = sm; sm *= s; }
        for (int n = m; n <= p; ++n) {
            long k = tri(n, m);
            out[k] = sm * Q[k];
            if (dtheta) dtheta[k] = (m == 0) ? -s * dQ[k] : smm1 * (m * t * Q[k] - s * s * dQ[k]);
            if (over_s) over_s[k] = (m == 0) ? 0.0 : smm1 * Q[k];
        }
    }
    free(Q);
    free(dQ);
}

/* Evaluate nf real fields (m >= 0 coefficients, packed per field) and, if
 * asked, d/dtheta and (1/sin theta) d/dphi, at the point with cos(theta)=t,
 * sin(theta)=s, longitude (cphi, sphi).  Work arrays Q, dQ of size tri(p+1,0). */
static void sh_point(int p, int nf, const double* coef, double t, double s, double cphi,
                     double sphi, int deriv, double* Q, double* dQ, double* val,
                     double* dth, double* dph)
{
    long nc = ncoef_of(p);
    leg_eval(p, t, Q, dQ);
    for (int f = 0; f < nf; ++f) { val[f] = 0.0; if (deriv) { dth[f] = 0.0; dph[f] = 0.0; } }
    double cm = 1.0, sm_ = 0.0;           /* cos(m phi), sin(m phi) */
    double pm = 1.0, pmm1 = 0.0;          /* s^m, s^(m-1) */
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            double c2 = cm * cphi - sm_ * sphi;
            double s2 = sm_ * cphi + cm * sphi;
            cm = c2;
            sm_ = s2;
            if (m == 1) { pmm1 = 1.0; pm = s; }
            else { pmm1 = pm; pm *= s; }
        }
        double mult = (m == 0) ? 1.0 : 2.0;
        for (int n = m; n <= p; ++n) {
            long k = tri(n, m);
            double P = pm * Q[k];
            double dP = (m == 0) ? -s * dQ[k] : pmm1 * (m * t * Q[k] - s * s * dQ[k]);
            double Ps = (m == 0) ? 0.0 : pmm1 * Q[k];
            for (int f = 0; f < nf; ++f) {
                double cr = coef[2 * (f * nc + k)], ci = coef[2 * (f * nc + k) + 1];
                double re = cr * cm - ci * sm_;           /* Re(c e^{im phi})      */
                val[f] += mult * re * P;
                if (deriv) {
                    dth[f] += mult * re * dP;
                    dph[f] += mult * (-(double)m) * (cr * sm_ + ci * cm) * Ps; /* Re(i m c e^{im phi}) */
                }
            }
        }
    }
}

/* Synthesis of nf degree-p fields on the degree-Q grid (values only), by
 * point evaluation.  out[f][j*nlon + k].                                    */
int ora_synth_grid(int p, int nf, const double* coef, int Q, int grid_mode, double* out)
{
    int nlat = Q + 1, nlon = nlon_of(Q, grid_mode);
    double* t = (double*)malloc(sizeof(double) * nlat);
    double* w = (double*)malloc(sizeof(double) * nlat);
    ora_gauss_legendre(nlat, t, w);
    long npts = (long)nlat * nlon;
#pragma omp parallel
    {
        long nc = ncoef_of(p);
        double* Qw = (double*)malloc(sizeof(double) * nc);
        double* dQw = (double*)malloc(sizeof(double) * nc);
        double* v = (double*)malloc(sizeof(double) * nf);
#pragma omp for schedule(static)
        for (long idx = 0; idx < npts; ++idx) {
            int j = (int)(idx / nlon), k = (int)(idx % nlon);
            double s = sqrt(1.0 - t[j] * t[j]);
            double ph = 2.0 * ORA_PI * k / nlon;
            sh_point(p, nf, coef, t[j], s, cos(ph), sin(ph), 0, Qw, dQw, v, NULL, NULL);
            for (int f = 0; f < nf; ++f) out[f * npts + idx] = v[f];
        }
        free(Qw); free(dQw); free(v);
    }
    free(t);
    free(w);
    return 0;
}

/* Galerkin analysis (y, Y_nm) = int y conj(Y_nm) ds on the unit sphere by the
 * grid quadrature, to degree p, from values on the degree-Q grid.          */
int ora_analyze_grid(int p, int nf, const double* grid, int Q, int grid_mode, double* coef)
{
    int nlat = Q + 1, nlon = nlon_of(Q, grid_mode);
    long nc = ncoef_of(p), npts = (long)nlat * nlon;
    double* t = (double*)malloc(sizeof(double) * nlat);
    double* w = (double*)malloc(sizeof(double) * nlat);
    ora_gauss_legendre(nlat, t, w);
    double* P = (double*)malloc(sizeof(double) * nc);
    memset(coef, 0, sizeof(double) * 2 * nc * nf);
    for (int j = 0; j < nlat; ++j) {
        double s = sqrt(1.0 - t[j] * t[j]);
        ora_pbar(p, t[j], s, P, NULL, NULL);
        for (int k = 0; k < nlon; ++k) {
            double ph = 2.0 * ORA_PI * k / nlon;
            double wt = 2.0 * ORA_PI / nlon * w[j];
            for (int f = 0; f < nf; ++f) {
                double y = grid[f * npts + (long)j * nlon + k];
                for (int n = 0; n <= p; ++n)
                    for (int m = 0; m <= n; ++m) {
                        long kk = tri(n, m);
                        coef[2 * (f * nc + kk)] += wt * y * P[kk] * cos(m * ph);
                        coef[2 * (f * nc + kk) + 1] -= wt * y * P[kk] * sin(m * ph);
                    }
            }
        }
    }
    free(P); free(t); free(w);
    return 0;
}

/* Evaluate a drop's position, tangent derivatives, normal and area factor
 * J = |x_theta x (x_phi / sin theta)| at one point.                          */
static void geom_point(int p, const double* xc, double t, double s, double cphi, double sphi,
                       double* Qw, double* dQw, double* x, double* nrm, double* J)
{
    double dth[3], dph[3];
    sh_point(p, 3, xc, t, s, cphi, sphi, 1, Qw, dQw, x, dth, dph);
    double cx = dth[1] * dph[2] - dth[2] * dph[1];
    double cy = dth[2] * dph[0] - dth[0] * dph[2];
    double cz = dth[0] * dph[1] - dth[1] * dph[0];
    double jj = sqrt(cx * cx + cy * cy + cz * cz);
    *J = jj;
    nrm[0] = cx / jj; nrm[1] = cy / jj; nrm[2] = cz / jj;
}

/* Add one source contribution (weight wq already contains the quadrature
 * weight and the area factor) to the 9 accumulators.                        */
static void kernel_add(const double* x0, const double* n0, const double* x, const double* n,
                       const double* f, const double* u, double sig, double wq, double* acc)
{
    double h[3] = { x0[0] - x[0], x0[1] - x[1], x0[2] - x[2] };  /* x-hat = x0 - x */
    double r2 = h[0] * h[0] + h[1] * h[1] + h[2] * h[2];
    double r = sqrt(r2);
    double ir = 1.0 / r, ir3 = ir / r2, ir5 = ir3 / r2;
    double hf = h[0] * f[0] + h[1] * f[1] + h[2] * f[2];
    double hu = h[0] * u[0] + h[1] * u[1] + h[2] * u[2];
    double hn = h[0] * n[0] + h[1] * n[1] + h[2] * n[2];
    double hn0 = h[0] * n0[0] + h[1] * n0[1] + h[2] * n0[2];
    for (int c = 0; c < 3; ++c) {
        acc[c] += wq * (f[c] * ir + h[c] * hf * ir3);          /* Stokeslet        */
        acc[3 + c] += wq * (-6.0 * hu * hn * ir5 * h[c]);       /* stresslet . n    */
    }
    acc[6] += wq * sig * ir;                                    /* Laplace SL       */
    acc[7] += wq * sig * hn * ir3;                              /* Laplace DL       */
    acc[8] += wq * sig * hn0 * ir3;                             /* adjoint DL       */
}

/* Drop table helper */
typedef struct {
    int nd;
    const int* p;
    long* off;           /* per-field double offsets */
} drops_t;

static void drops_init(drops_t* d, int nd, const int* p)
{
    d->nd = nd;
    d->p = p;
    d->off = (long*)malloc(sizeof(long) * (nd + 1));
    d->off[0] = 0;
    for (int i = 0; i < nd; ++i) d->off[i + 1] = d->off[i] + (long)(p[i] + 1) * (p[i] + 2);
}

/* Target positions and normals at the drops' own degree-p grid nodes.
 * tgt_node = j*nlon + k.                                                    */
int ora_targets(int nd, const int* p, int grid_mode, const double* xcoef, int nt,
                const int* tgt_drop, const int* tgt_node, double* x0 /*[3][nt]*/,
                double* n0 /*[3][nt]*/)
{
    drops_t D;
    drops_init(&D, nd, p);
    int pmax = 0;
    for (int i = 0; i < nd; ++i) if (p[i] > pmax) pmax = p[i];
#pragma omp parallel
    {
        long nc = ncoef_of(pmax);
        double* Qw = (double*)malloc(sizeof(double) * nc);
        double* dQw = (double*)malloc(sizeof(double) * nc);
        double* tt = (double*)malloc(sizeof(double) * (pmax + 1));
        double* ww = (double*)malloc(sizeof(double) * (pmax + 1));
#pragma omp for schedule(dynamic, 16)
        for (int it = 0; it < nt; ++it) {
            int d = tgt_drop[it], pd = p[d];
            int nlon = nlon_of(pd, grid_mode);
            int j = tgt_node[it] / nlon, k = tgt_node[it] % nlon;
            ora_gauss_legendre(pd + 1, tt, ww);
            double s = sqrt(1.0 - tt[j] * tt[j]);
            double ph = 2.0 * ORA_PI * k / nlon;
            double xx[3], nn[3], J;
            geom_point(pd, xcoef + 3 * D.off[d], tt[j], s, cos(ph), sin(ph), Qw, dQw, xx, nn, &J);
            for (int c = 0; c < 3; ++c) { x0[c * nt + it] = xx[c]; n0[c * nt + it] = nn[c]; }
        }
        free(Qw); free(dQw); free(tt); free(ww);
    }
    free(D.off);
    return 0;
}

/* Far field: for each target point (x0, n0) sum the regular quadrature
 * (eq. reg_quadrature) over the degree-qfar grid of every drop except
 * tgt_exclude[i] (-1: none).  Sources are built once by point evaluation.   */
/* Source records of the regular rule (eq. reg_quadrature) on every drop's
 * degree-qfar grid: x(3) n(3) f(3) u(3) sigma(1) weight(1) per node.  The
 * returned block holds the node offsets of the drops (nd + 1 longs) and then
 * the records; ora_far_free releases it.                                    */
typedef struct {
    int nd;
    long* soff;
    double* src;
} far_src_t;

void* ora_far_sources(int nd, const int* p, const int* qfar, int grid_mode, const double* xcoef,
                      const double* fcoef, const double* ucoef, const double* sigcoef)
{
    drops_t D;
    drops_init(&D, nd, p);
    long* soff = (long*)malloc(sizeof(long) * (nd + 1));
    soff[0] = 0;
    for (int d = 0; d < nd; ++d)
        soff[d + 1] = soff[d] + (long)(qfar[d] + 1) * nlon_of(qfar[d], grid_mode);
    long ns = soff[nd];
    /* source record: x(3) n(3) f(3) u(3) sigma(1) weight(1) */
    double* src = (double*)malloc(sizeof(double) * 14 * ns);
    int pmax = 0;
    for (int i = 0; i < nd; ++i) if (p[i] > pmax) pmax = p[i];
    for (int d = 0; d < nd; ++d) {
        int Q = qfar[d], nlat = Q + 1, nlon = nlon_of(Q, grid_mode);
        double* tt = (double*)malloc(sizeof(double) * nlat);
        double* ww = (double*)malloc(sizeof(double) * nlat);
        ora_gauss_legendre(nlat, tt, ww);
        long nc = ncoef_of(p[d]);
        const double* xc = xcoef + 3 * D.off[d];
        const double* fc = fcoef + 3 * D.off[d];
        const double* uc = ucoef ? ucoef + 3 * D.off[d] : fc;
        const double* sc = sigcoef + D.off[d];
#pragma omp parallel
        {
            double* Qw = (double*)malloc(sizeof(double) * ncoef_of(pmax));
            double* dQw = (double*)malloc(sizeof(double) * ncoef_of(pmax));
#pragma omp for schedule(static)
            for (long idx = 0; idx < (long)nlat * nlon; ++idx) {
                int j = (int)(idx / nlon), k = (int)(idx % nlon);
                double s = sqrt(1.0 - tt[j] * tt[j]);
                double ph = 2.0 * ORA_PI * k / nlon;
                double cph = cos(ph), sph = sin(ph);
                double* r = src + 14 * (soff[d] + idx);
                double J;
                geom_point(p[d], xc, tt[j], s, cph, sph, Qw, dQw, r, r + 3, &J);
                sh_point(p[d], 3, fc, tt[j], s, cph, sph, 0, Qw, dQw, r + 6, NULL, NULL);
                sh_point(p[d], 3, uc, tt[j], s, cph, sph, 0, Qw, dQw, r + 9, NULL, NULL);
                sh_point(p[d], 1, sc, tt[j], s, cph, sph, 0, Qw, dQw, r + 12, NULL, NULL);
                r[13] = 2.0 * ORA_PI / nlon * ww[j] * J;
            }
            free(Qw); free(dQw);
        }
        (void)nc;
        free(tt); free(ww);
    }
    free(D.off);
    far_src_t* h = (far_src_t*)malloc(sizeof(far_src_t));
    h->nd = nd;
    h->soff = soff;
    h->src = src;
    return h;
}

void ora_far_free(void* handle)
{
    far_src_t* h = (far_src_t*)handle;
    if (!h) return;
    free(h->src);
    free(h->soff);
    free(h);
}

/* Far-field sums at arbitrary points x0 with target normals n0: every
 * drop's records except the drop tgt_exclude[it] (NULL: none), natural
 * order, times 1/(4 pi).                                                    */
int ora_far_eval(const void* handle, int nt, const double* x0 /*[3][nt]*/, const double* n0 /*[3][nt]*/,
                 const int* tgt_exclude, double* out /*[9][nt]*/)
{
    const far_src_t* h = (const far_src_t*)handle;
    const int nd = h->nd;
    const long* soff = h->soff;
    const double* src = h->src;
#pragma omp parallel for schedule(dynamic, 8)
    for (int it = 0; it < nt; ++it) {
        double acc[NCOMP] = {0};
        double xx[3] = { x0[it], x0[nt + it], x0[2 * nt + it] };
        double nn[3] = { n0[it], n0[nt + it], n0[2 * nt + it] };
        int ex = tgt_exclude ? tgt_exclude[it] : -1;
        for (int d = 0; d < nd; ++d) {
            if (d == ex) continue;
            for (long is = soff[d]; is < soff[d + 1]; ++is) {
                const double* r = src + 14 * is;
                kernel_add(xx, nn, r, r + 3, r + 6, r + 9, r[12], r[13], acc);
            }
        }
        for (int c = 0; c < NCOMP; ++c) out[c * nt + it] = acc[c] / (4.0 * ORA_PI);
    }
    return 0;
}

int ora_far(int nd, const int* p, const int* qfar, int grid_mode, const double* xcoef,
            const double* fcoef, const double* ucoef, const double* sigcoef, int nt,
            const double* x0 /*[3][nt]*/, const double* n0 /*[3][nt]*/,
            const int* tgt_exclude, double* out /*[9][nt]*/)
{
    void* h = ora_far_sources(nd, p, qfar, grid_mode, xcoef, fcoef, ucoef, sigcoef);
    int rc = ora_far_eval(h, nt, x0, n0, tgt_exclude, out);
    ora_far_free(h);
    return rc;
}

/* Sum_{n=0}^{N} P_n(t) by the Legendre recurrence. */
static double legendre_sum(int N, double t)
{
    double pkm1 = 1.0, pk = t, sum = 1.0;
    if (N >= 1) sum += t;
    for (int k = 1; k < N; ++k) {
        double pkp1 = ((2.0 * k + 1.0) * t * pk - k * pkm1) / (k + 1.0);
        pkm1 = pk;
        pk = pkp1;
        sum += pk;
    }
    return sum;
}

/* Singular self-interaction at targets (drop, node j*nlon+k of its degree-p
 * grid), eq. mod_weights with the target rotated to the north pole.
 * For each target the degree-qself Gaussian grid (theta', phi') is laid out
 * around the pole, each node s' is mapped to s = Rz(phi_t) Ry(theta_t) s',
 * and the drop's own (unrotated) expansions are evaluated at s.             */
int ora_self(int nd, const int* p, const int* qself, int grid_mode, const double* xcoef,
             const double* fcoef, const double* ucoef, const double* sigcoef, int nt,
             const int* tgt_drop, const int* tgt_node, double* out /*[9][nt]*/)
{
    drops_t D;
    drops_init(&D, nd, p);
    int pmax = 0, qmax = 0;
    for (int i = 0; i < nd; ++i) { if (p[i] > pmax) pmax = p[i]; if (qself[i] > qmax) qmax = qself[i]; }
#pragma omp parallel
    {
        long nc = ncoef_of(pmax);
        double* Qw = (double*)malloc(sizeof(double) * nc);
        double* dQw = (double*)malloc(sizeof(double) * nc);
        double* tp = (double*)malloc(sizeof(double) * (pmax + 1));
        double* wp = (double*)malloc(sizeof(double) * (pmax + 1));
        double* tq = (double*)malloc(sizeof(double) * (qmax + 1));
        double* wq = (double*)malloc(sizeof(double) * (qmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int it = 0; it < nt; ++it) {
            int d = tgt_drop[it], pd = p[d], Q = qself[d];
            int nlon = nlon_of(pd, grid_mode), nlonq = nlon_of(Q, grid_mode);
            int j = tgt_node[it] / nlon, k = tgt_node[it] % nlon;
            const double* xc = xcoef + 3 * D.off[d];
            const double* fc = fcoef + 3 * D.off[d];
            const double* uc = ucoef ? ucoef + 3 * D.off[d] : fc;
            const double* sc = sigcoef + D.off[d];
            ora_gauss_legendre(pd + 1, tp, wp);
            ora_gauss_legendre(Q + 1, tq, wq);
            double ct = tp[j], st = sqrt(1.0 - ct * ct);
            double pht = 2.0 * ORA_PI * k / nlon, cpt = cos(pht), spt = sin(pht);
            double x0[3], n0[3], J0;
            geom_point(pd, xc, ct, st, cpt, spt, Qw, dQw, x0, n0, &J0);
            double acc[NCOMP] = {0};
            for (int i = 0; i < Q + 1; ++i) {
                double si = sqrt(1.0 - tq[i] * tq[i]);
                double wmod = 2.0 * ORA_PI / nlonq * wq[i] * sqrt(2.0 - 2.0 * tq[i]) *
                              legendre_sum(Q, tq[i]);
                for (int l = 0; l < nlonq; ++l) {
                    double phl = 2.0 * ORA_PI * l / nlonq;
                    double v[3] = { si * cos(phl), si * sin(phl), tq[i] };
                    /* Ry(theta_t) */
                    double a[3] = { ct * v[0] + st * v[2], v[1], -st * v[0] + ct * v[2] };
                    /* Rz(phi_t) */
                    double sv[3] = { cpt * a[0] - spt * a[1], spt * a[0] + cpt * a[1], a[2] };
                    double s = sqrt(sv[0] * sv[0] + sv[1] * sv[1]);
                    double cph = 1.0, sph = 0.0;
                    if (s > 0.0) { cph = sv[0] / s; sph = sv[1] / s; }
                    double tt = sv[2];
                    double xx[3], nn[3], J, ff[3], uu[3], sg;
                    geom_point(pd, xc, tt, s, cph, sph, Qw, dQw, xx, nn, &J);
                    sh_point(pd, 3, fc, tt, s, cph, sph, 0, Qw, dQw, ff, NULL, NULL);
                    sh_point(pd, 3, uc, tt, s, cph, sph, 0, Qw, dQw, uu, NULL, NULL);
                    sh_point(pd, 1, sc, tt, s, cph, sph, 0, Qw, dQw, &sg, NULL, NULL);
                    kernel_add(x0, n0, xx, nn, ff, uu, sg, wmod * J, acc);
                }
            }
            for (int c = 0; c < NCOMP; ++c) out[c * nt + it] = acc[c] / (4.0 * ORA_PI);
        }
        free(Qw); free(dQw); free(tp); free(wp); free(tq); free(wq);
    }
    free(D.off);
    return 0;
}

/* Regular quadrature of a scalar field g (given by SH coefficients, degree
 * pg) over drop surface x (degree p) on the degree-Q grid: int g dS.  Also
 * returns the enclosed volume (1/3) int x.n dS and the area.               */
int ora_surface_integrals(int p, const double* xcoef, int pg, const double* gcoef, int Q,
                          int grid_mode, double* area, double* volume, double* gint)
{
    int nlat = Q + 1, nlon = nlon_of(Q, grid_mode);
    int pm = p > pg ? p : pg;
    double* t = (double*)malloc(sizeof(double) * nlat);
    double* w = (double*)malloc(sizeof(double) * nlat);
    double* Qw = (double*)malloc(sizeof(double) * ncoef_of(pm));
    double* dQw = (double*)malloc(sizeof(double) * ncoef_of(pm));
    ora_gauss_legendre(nlat, t, w);
    double A = 0.0, V = 0.0, G = 0.0;
    for (int j = 0; j < nlat; ++j) {
        double s = sqrt(1.0 - t[j] * t[j]);
        for (int k = 0; k < nlon; ++k) {
            double ph = 2.0 * ORA_PI * k / nlon;
            double xx[3], nn[3], J, g = 0.0;
            geom_point(p, xcoef, t[j], s, cos(ph), sin(ph), Qw, dQw, xx, nn, &J);
            if (gcoef) sh_point(pg, 1, gcoef, t[j], s, cos(ph), sin(ph), 0, Qw, dQw, &g, NULL, NULL);
            double wt = 2.0 * ORA_PI / nlon * w[j] * J;
            A += wt;
            V += wt * (xx[0] * nn[0] + xx[1] * nn[1] + xx[2] * nn[2]) / 3.0;
            G += wt * g;
        }
    }
    *area = A; *volume = V; *gint = G;
    free(t); free(w); free(Qw); free(dQw);
    return 0;
}

/* Point evaluation exposed for the pins: values, d/dtheta, (1/s) d/dphi. */
void ora_sh_point(int p, int nf, const double* coef, double t, double s, double cphi,
                  double sphi, double* val, double* dth, double* dph)
{
    double* Qw = (double*)malloc(sizeof(double) * ncoef_of(p));
    double* dQw = (double*)malloc(sizeof(double) * ncoef_of(p));
    sh_point(p, nf, coef, t, s, cphi, sphi, 1, Qw, dQw, val, dth, dph);
    free(Qw); free(dQw);
}

/* Geometry at a point (x, n, J) exposed for the pins. */
void ora_geom_point(int p, const double* xcoef, double t, double s, double cphi, double sphi,
                    double* x, double* n, double* J)
{
    double* Qw = (double*)malloc(sizeof(double) * ncoef_of(p));
    double* dQw = (double*)malloc(sizeof(double) * ncoef_of(p));
    geom_point(p, xcoef, t, s, cphi, sphi, Qw, dQw, x, n, J);
    free(Qw); free(dQw);
}

/* Q, dQ/dt and d2Q/dt2 of Pbar_n^m = s^m Q(t) by the recurrence in n and
 * its first and second t-derivatives. */
static void leg_eval2(int p, double t, double* Q, double* dQ, double* d2Q)
{
    double qmm = 1.0 / sqrt(4.0 * ORA_PI);
    for (int m = 0; m <= p; ++m) {
        if (m > 0) qmm *= -sqrt((2.0 * m + 1.0) / (2.0 * m));
        Q[tri(m, m)] = qmm;
        dQ[tri(m, m)] = 0.0;
        d2Q[tri(m, m)] = 0.0;
        if (m + 1 <= p) {
            double c = sqrt(2.0 * m + 3.0);
            Q[tri(m + 1, m)] = c * t * qmm;
            dQ[tri(m + 1, m)] = c * qmm;
            d2Q[tri(m + 1, m)] = 0.0;
        }
        for (int n = m + 2; n <= p; ++n) {
            double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
            double b = sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
            long k = tri(n, m), k1 = tri(n - 1, m), k2 = tri(n - 2, m);
            Q[k] = a * (t * Q[k1] - b * Q[k2]);
            dQ[k] = a * (Q[k1] + t * dQ[k1] - b * dQ[k2]);
            d2Q[k] = a * (2.0 * dQ[k1] + t * d2Q[k1] - b * d2Q[k2]);
        }
    }
}

/* Surface quantities at the point (theta, phi) of a drop x (3 fields) and of
 * ng scalar fields g (packed, degree p):
 *   out[0..2] x, out[3..5] n (outward unit normal), out[6] mean curvature
 *   H = (1/2) div_S n (Sec. 1, after eq. interfacial_force), out[7 + 4 g ..]
 *   the surface gradient of field g (3) and its Laplace-Beltrami (1),
 *   Lap_S g = g^{ij} (g_{,ij} - x_{,ij} . grad_S g), the trace of the
 *   surface Hessian (Christoffel terms x_{,ij} . x^{,k} g_{,k}).
 * With x_a, x_ab the parameter derivatives, E, F, G and L, M, N the first
 * and second fundamental forms (L = x_tt . n, ...), W^2 = EG - F^2:
 *   H = -(E N - 2 F M + G L) / (2 W^2)   (positive on a sphere with outward n),
 *   grad_S g = ((G g_t - F g_p) x_t + (E g_p - F g_t) x_p) / W^2.
 * Derivatives of Pbar = s^m Q(t), t = cos theta, s = sin theta:
 *   d/dtheta   = m s^(m-1) t Q - s^(m+1) Q',
 *   d2/dtheta2 = m(m-1) s^(m-2) t^2 Q - m s^m Q - (2m+1) s^m t Q' + s^(m+2) Q''. */
void ora_surface_point(int p, const double* xcoef, int ng, const double* gcoef, double theta, double phi,
                       double* out)
{
    long nc = ncoef_of(p);
    double* Q = (double*)malloc(sizeof(double) * nc);
    double* dQ = (double*)malloc(sizeof(double) * nc);
    double* d2Q = (double*)malloc(sizeof(double) * nc);
    double t = cos(theta), s = sin(theta);
    leg_eval2(p, t, Q, dQ, d2Q);
    int nf = 3 + ng;
    double v[64], vt[64], vp[64], vtt[64], vtp[64], vpp[64];
    for (int f = 0; f < nf; ++f) { v[f] = vt[f] = vp[f] = 0.0; vtt[f] = vtp[f] = vpp[f] = 0.0; }
    for (int m = 0; m <= p; ++m) {
        double cm = cos(m * phi), sm_ = sin(m * phi);
        double mult = (m == 0) ? 1.0 : 2.0;
        double sm0 = pow(s, m), sm1 = m >= 1 ? pow(s, m - 1) : 0.0, sm2 = m >= 2 ? pow(s, m - 2) : 0.0;
        for (int n = m; n <= p; ++n) {
            long k = tri(n, m);
            double P = sm0 * Q[k];
            double dP = m * sm1 * t * Q[k] - sm0 * s * dQ[k];
            double d2P = m * (m - 1) * sm2 * t * t * Q[k] - m * sm0 * Q[k] - (2.0 * m + 1.0) * sm0 * t * dQ[k] +
                         sm0 * s * s * d2Q[k];
            for (int f = 0; f < nf; ++f) {
                const double* cf = f < 3 ? xcoef + 2 * (f * nc + k) : gcoef + 2 * ((f - 3) * nc + k);
                double cr = cf[0], ci = (m == 0) ? 0.0 : cf[1];
                double re = cr * cm - ci * sm_;          /* Re(c e^{i m phi})   */
                double im = cr * sm_ + ci * cm;          /* Im(c e^{i m phi})   */
                v[f] += mult * re * P;
                vt[f] += mult * re * dP;
                vp[f] += mult * (-(double)m) * im * P;   /* d/dphi: Re(i m c e^{i m phi}) */
                vtt[f] += mult * re * d2P;
                vtp[f] += mult * (-(double)m) * im * dP;
                vpp[f] += mult * (-(double)m * m) * re * P;
            }
        }
    }
    double E = 0, F = 0, G = 0;
    for (int c = 0; c < 3; ++c) { E += vt[c] * vt[c]; F += vt[c] * vp[c]; G += vp[c] * vp[c]; }
    double nx = vt[1] * vp[2] - vt[2] * vp[1], ny = vt[2] * vp[0] - vt[0] * vp[2], nz = vt[0] * vp[1] - vt[1] * vp[0];
    double W = sqrt(nx * nx + ny * ny + nz * nz);
    nx /= W; ny /= W; nz /= W;
    double L = vtt[0] * nx + vtt[1] * ny + vtt[2] * nz;
    double M = vtp[0] * nx + vtp[1] * ny + vtp[2] * nz;
    double N = vpp[0] * nx + vpp[1] * ny + vpp[2] * nz;
    double W2 = E * G - F * F;
    for (int c = 0; c < 3; ++c) out[c] = v[c];
    out[3] = nx; out[4] = ny; out[5] = nz;
    out[6] = -(E * N - 2.0 * F * M + G * L) / (2.0 * W2);
    for (int g = 0; g < ng; ++g) {
        double gt = vt[3 + g], gp = vp[3 + g];
        double a = (G * gt - F * gp) / W2, b = (E * gp - F * gt) / W2;
        double gr[3];
        for (int c = 0; c < 3; ++c) {
            gr[c] = a * vt[c] + b * vp[c];
            out[7 + 4 * g + c] = gr[c];
        }
        double htt = vtt[3 + g], htp = vtp[3 + g], hpp = vpp[3 + g];
        for (int c = 0; c < 3; ++c) {
            htt -= vtt[c] * gr[c];
            htp -= vtp[c] * gr[c];
            hpp -= vpp[c] * gr[c];
        }
        out[7 + 4 * g + 3] = (G * htt - 2.0 * F * htp + E * hpp) / W2;
    }
    free(Q); free(dQ); free(d2Q);
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of OpenMP threads of later calls (n >= 1). */
void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
