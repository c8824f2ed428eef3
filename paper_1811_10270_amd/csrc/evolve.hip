// Time stepping of the drops and their surfactant (Sec. 2.2, Algorithm 1):
// the midpoint rule for the surfaces and the second-order implicit-explicit
// Runge-Kutta scheme for the surfactant (implicit surface diffusion,
// explicit convection), with the error estimate and step-size rule of the
// algorithm's adaptivity part.  Every stage runs through the library's
// device entry points (solvers, surface quantities, projection); this file
// adds the convective term, the stage arithmetic and the step control.
//
// Surface points move with the full velocity u (x' = u).  Following those
// points, eq. surfactant0 reads dGamma/dt = -Gamma div_S u + Pe^-1 Lap_S Gamma
// (its terms div_S(Gamma u_t) + 2 H Gamma (u.n) plus the frame term
// u_t . grad_S Gamma; div_S u = div_S u_t + 2 H u.n with H = div_S n / 2),
// so the convective part is g_E = -Gamma div_S u and the diffusive part
// g_I = Pe^-1 Lap_S Gamma; with it d/dt (Gamma dA) = Pe^-1 Lap_S Gamma dA and
// the surfactant mass is conserved.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "ctx_access.h"
#include "ehdbim.h"

namespace {

constexpr int kT = 256;
unsigned nblk(long long n) { return (unsigned)((n + kT - 1) / kT); }

// out = -Gamma div_S u, div_S u = sum_c (grad_S u_c)_c; grad[c][k][T]
__global__ void k_conv_term(const double* __restrict__ grad, const double* __restrict__ G, long long T,
                            double* __restrict__ out)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const double div = grad[t] + grad[4 * T + t] + grad[8 * T + t];
    out[t] = -G[t] * div;
}

// z = a x + b y
__global__ void k_lin2(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                       double* __restrict__ z, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) z[t] = a * x[t] + b * y[t];
}

// x *= a
__global__ void k_scale(double a, double* __restrict__ x, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] *= a;
}

// z = x + a (y1 + y2)
__global__ void k_add2(const double* __restrict__ x, double a, const double* __restrict__ y1,
                       const double* __restrict__ y2, double* __restrict__ z, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) z[t] = x[t] + a * (y1[t] + y2[t]);
}

// z = (x1 + x2) - (y1 + y2)
__global__ void k_diff2(const double* __restrict__ x1, const double* __restrict__ x2, const double* __restrict__ y1,
                        const double* __restrict__ y2, double* __restrict__ z, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) z[t] = (x1[t] + x2[t]) - (y1[t] + y2[t]);
}

// per-block maxima of |x|
__global__ __launch_bounds__(kT) void k_absmax(const double* __restrict__ x, long long n, double* __restrict__ part)
{
    __shared__ double sh[kT];
    double m = 0.0;
    for (long long t = (long long)blockIdx.x * kT + threadIdx.x; t < n; t += (long long)gridDim.x * kT)
        m = fmax(m, fabs(x[t]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

#define EVO_HIP(call)                                                                                \
    do {                                                                                             \
        hipError_t _e = (call);                                                                      \
        if (_e != hipSuccess) {                                                                      \
            char _b[256];                                                                            \
            snprintf(_b, sizeof(_b), "%s failed: %s", #call, hipGetErrorString(_e));                 \
            return ehd_ctx_fail(ctx, EHD_E_HIP, _b);                                                 \
        }                                                                                            \
    } while (0)

struct Buf {
    double* p = nullptr;
    ~Buf()
    {
        if (p) (void)hipFree(p);
    }
};

// Device work space of one stepping call.
struct Work {
    long long T = 0, nc = 0;
    Buf H, grad3, lap, gv, val, xdum, part, xn;
    Buf enA, uA, gEA, gIA;        // stage at (x^n, Gamma^n)
    Buf enB, uB, gEB, gIB;        // stage at the half step
    Buf xh, Gh, rhs;
    Buf d3, dv;                   // error-estimate scratch: 3 fields of coefficients, of node values
    static constexpr int kParts = 64;
};

int alloc(ehd_ctx* ctx, Buf& b, long long n)
{
    EVO_HIP(hipMalloc(&b.p, sizeof(double) * (size_t)std::max(n, 1LL)));
    return EHD_OK;
}

int make_work(ehd_ctx* ctx, Work& w)
{
    int rc;
    if ((rc = ehd_num_targets(ctx, &w.T)) || (rc = ehd_num_coefs(ctx, &w.nc))) return rc;
    const long long T = w.T, nc = w.nc;
    Buf* tl[] = {&w.H, &w.lap, &w.gv, &w.val};
    for (Buf* b : tl)
        if ((rc = alloc(ctx, *b, T))) return rc;
    if ((rc = alloc(ctx, w.grad3, 9 * T)) || (rc = alloc(ctx, w.part, Work::kParts)) ||
        (rc = alloc(ctx, w.d3, 3 * nc)) || (rc = alloc(ctx, w.dv, 3 * T)))
        return rc;
    Buf* c3[] = {&w.xdum, &w.xn, &w.uA, &w.uB, &w.xh};
    for (Buf* b : c3)
        if ((rc = alloc(ctx, *b, 3 * nc))) return rc;
    Buf* c1[] = {&w.enA, &w.gEA, &w.gIA, &w.enB, &w.gEB, &w.gIB, &w.Gh, &w.rhs};
    for (Buf* b : c1)
        if ((rc = alloc(ctx, *b, nc))) return rc;
    EVO_HIP(hipMemsetAsync(w.enA.p, 0, sizeof(double) * nc, ehd_ctx_stream(ctx)));
    EVO_HIP(hipMemsetAsync(w.uA.p, 0, sizeof(double) * 3 * nc, ehd_ctx_stream(ctx)));
    return EHD_OK;
}

// max |x| over n device values (synchronous)
int absmax(ehd_ctx* ctx, Work& w, const double* x, long long n, double* out)
{
    hipStream_t st = ehd_ctx_stream(ctx);
    const int nb = (int)std::min<long long>(Work::kParts, std::max<long long>(1, (n + kT - 1) / kT));
    hipLaunchKernelGGL(k_absmax, dim3(nb), dim3(kT), 0, st, x, n, w.part.p);
    EVO_HIP(hipGetLastError());
    double h[Work::kParts];
    EVO_HIP(hipMemcpyAsync(h, w.part.p, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    EVO_HIP(hipStreamSynchronize(st));
    double m = 0.0;
    for (int i = 0; i < nb; ++i) m = std::max(m, h[i]);
    *out = m;
    return EHD_OK;
}

// g_E = P[-Gamma div_S u] and g_I = P[inv_pe Lap_S Gamma] on the current surfaces
int surf_terms(ehd_ctx* ctx, Work& w, const double* u, const double* G, double inv_pe, double* gE, double* gI)
{
    hipStream_t st = ehd_ctx_stream(ctx);
    int rc;
    if (gE) {
        if ((rc = ehd_surface(ctx, 3, u, w.H.p, w.grad3.p, nullptr))) return rc;
        if ((rc = ehd_synthesize(ctx, 1, G, w.gv.p))) return rc;
        hipLaunchKernelGGL(k_conv_term, dim3(nblk(w.T)), dim3(kT), 0, st, w.grad3.p, w.gv.p, w.T, w.val.p);
        EVO_HIP(hipGetLastError());
        if ((rc = ehd_analyze(ctx, 1, w.val.p, gE))) return rc;
    }
    if (gI) {
        if ((rc = ehd_surface(ctx, 1, G, w.H.p, w.grad3.p, w.lap.p))) return rc;
        if ((rc = ehd_analyze(ctx, 1, w.lap.p, gI))) return rc;
        hipLaunchKernelGGL(k_scale, dim3(nblk(w.nc)), dim3(kT), 0, st, inv_pe, gI, w.nc);
        EVO_HIP(hipGetLastError());
    }
    return EHD_OK;
}

// Velocity stage on the current surfaces: E_n, forces, u (guesses in en, u).
int velocity_stage(ehd_ctx* ctx, Work& w, const ehd_step_params* prm, const double* G, double* en, double* u,
                   int* its)
{
    ehd_step_params q = *prm;
    q.dt = 0.0;
    return ehd_explicit_step(ctx, &q, G, en, u, w.xdum.p, its);
}

int check_params(ehd_ctx* ctx, const ehd_step_params* prm, double inv_pe)
{
    if (!prm) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL parameters");
    if (!(inv_pe >= 0.0) || !std::isfinite(inv_pe)) return ehd_ctx_fail(ctx, EHD_E_ARG, "inv_pe must be >= 0");
    return EHD_OK;
}

// The state-dependent first stage: u^n, g_E^n, g_I^n at (x^n, Gamma^n).
int stage_a(ehd_ctx* ctx, Work& w, const ehd_step_params* prm, double inv_pe, const double* G0, int* its)
{
    int rc = velocity_stage(ctx, w, prm, G0, w.enA.p, w.uA.p, its);
    if (!rc) rc = surf_terms(ctx, w, w.uA.p, G0, inv_pe, w.gEA.p, w.gIA.p);
    return rc;
}

// One step of size dt from (x^n in w.xn, Gamma^n in G0) after stage_a.
// Leaves the context on the half-step surface.  Proposals into xnew, gnew.
int step_b(ehd_ctx* ctx, Work& w, const ehd_step_params* prm, double inv_pe, double dt, const double* G0,
           double* xnew, double* gnew, ehd_step_report* rep)
{
    hipStream_t st = ehd_ctx_stream(ctx);
    const long long nc = w.nc, T = w.T;
    int rc;
    // x^{n+1/2} = x^n + dt/2 u^n
    hipLaunchKernelGGL(k_lin2, dim3(nblk(3 * nc)), dim3(kT), 0, st, 1.0, w.xn.p, 0.5 * dt, w.uA.p, w.xh.p, 3 * nc);
    EVO_HIP(hipGetLastError());
    if ((rc = ehd_update_shape(ctx, w.xh.p))) return rc;
    // (I - dt/(2 Pe) Lap_S) Gamma^{n+1/2} = Gamma^n + dt/2 g_E^n on the half-step surfaces
    hipLaunchKernelGGL(k_lin2, dim3(nblk(nc)), dim3(kT), 0, st, 1.0, G0, 0.5 * dt, w.gEA.p, w.rhs.p, nc);
    EVO_HIP(hipGetLastError());
    EVO_HIP(hipMemcpyAsync(w.Gh.p, G0, sizeof(double) * nc, hipMemcpyDeviceToDevice, st));
    rep->iters_gamma = 0;
    if (inv_pe > 0.0) {
        std::vector<double> kap(ehd_ctx_ndrops(ctx), 0.5 * dt * inv_pe);
        double rr;
        if ((rc = ehd_solve_surfactant(ctx, kap.data(), w.rhs.p, 1, prm->restart, prm->maxit, prm->tol, w.Gh.p,
                                       &rep->iters_gamma, &rr)))
            return rc;
    } else {
        EVO_HIP(hipMemcpyAsync(w.Gh.p, w.rhs.p, sizeof(double) * nc, hipMemcpyDeviceToDevice, st));
    }
    // u^{n+1/2}, g_E and g_I at the half step
    EVO_HIP(hipMemcpyAsync(w.enB.p, w.enA.p, sizeof(double) * nc, hipMemcpyDeviceToDevice, st));
    EVO_HIP(hipMemcpyAsync(w.uB.p, w.uA.p, sizeof(double) * 3 * nc, hipMemcpyDeviceToDevice, st));
    if ((rc = velocity_stage(ctx, w, prm, w.Gh.p, w.enB.p, w.uB.p, rep->iters + 2))) return rc;
    if ((rc = surf_terms(ctx, w, w.uB.p, w.Gh.p, inv_pe, w.gEB.p, w.gIB.p))) return rc;
    // x^{n+1} = x^n + dt u^{n+1/2}; Gamma^{n+1} = Gamma^n + dt (g_E + g_I)^{n+1/2}
    hipLaunchKernelGGL(k_lin2, dim3(nblk(3 * nc)), dim3(kT), 0, st, 1.0, w.xn.p, dt, w.uB.p, xnew, 3 * nc);
    hipLaunchKernelGGL(k_add2, dim3(nblk(nc)), dim3(kT), 0, st, G0, dt, w.gEB.p, w.gIB.p, gnew, nc);
    EVO_HIP(hipGetLastError());
    // error estimates: differences to the first-order updates from the
    // first stage, x^n + dt u^n and Gamma^n + dt (g_E + g_I)^n, at the nodes
    hipLaunchKernelGGL(k_lin2, dim3(nblk(3 * nc)), dim3(kT), 0, st, dt, w.uB.p, -dt, w.uA.p, w.d3.p, 3 * nc);
    EVO_HIP(hipGetLastError());
    if ((rc = ehd_synthesize(ctx, 3, w.d3.p, w.dv.p))) return rc;
    if ((rc = absmax(ctx, w, w.dv.p, 3 * T, &rep->err_drop))) return rc;
    hipLaunchKernelGGL(k_diff2, dim3(nblk(nc)), dim3(kT), 0, st, w.gEB.p, w.gIB.p, w.gEA.p, w.gIA.p, w.d3.p, nc);
    EVO_HIP(hipGetLastError());
    if ((rc = ehd_synthesize(ctx, 1, w.d3.p, w.dv.p))) return rc;
    double e;
    if ((rc = absmax(ctx, w, w.dv.p, T, &e))) return rc;
    rep->err_surf = dt * e;
    return EHD_OK;
}

}  // namespace

extern "C" {

int ehd_surfactant_terms(ehd_ctx* ctx, const double* ucoef_d, const double* gamma_d, double inv_pe, double* gE_d,
                         double* gI_d)
{
    if (!ctx) return EHD_E_ARG;
    if (!ehd_ctx_ndrops(ctx)) return ehd_ctx_fail(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!gamma_d || (gE_d && !ucoef_d)) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL argument");
    if (!(inv_pe >= 0.0) || !std::isfinite(inv_pe)) return ehd_ctx_fail(ctx, EHD_E_ARG, "inv_pe must be >= 0");
    EVO_HIP(hipSetDevice(ehd_ctx_device(ctx)));
    Work w;
    int rc = make_work(ctx, w);
    if (!rc) rc = surf_terms(ctx, w, ucoef_d, gamma_d, inv_pe, gE_d, gI_d);
    if (!rc) EVO_HIP(hipStreamSynchronize(ehd_ctx_stream(ctx)));
    return rc;
}

int ehd_evolve_step(ehd_ctx* ctx, const ehd_step_params* prm, double inv_pe, double dt, const double* gamma_d,
                    double* xnew_d, double* gnew_d, ehd_step_report* rep)
{
    if (!ctx) return EHD_E_ARG;
    if (!ehd_ctx_ndrops(ctx)) return ehd_ctx_fail(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!gamma_d || !xnew_d || !gnew_d || !rep) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL argument");
    int rc = check_params(ctx, prm, inv_pe);
    if (rc) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return ehd_ctx_fail(ctx, EHD_E_ARG, "dt must be > 0");
    *rep = ehd_step_report{};
    EVO_HIP(hipSetDevice(ehd_ctx_device(ctx)));
    Work w;
    if ((rc = make_work(ctx, w))) return rc;
    if ((rc = ehd_drop_coefs(ctx, w.xn.p))) return rc;
    if ((rc = stage_a(ctx, w, prm, inv_pe, gamma_d, rep->iters))) return rc;
    rc = step_b(ctx, w, prm, inv_pe, dt, gamma_d, xnew_d, gnew_d, rep);
    const int rc2 = ehd_update_shape(ctx, w.xn.p);       // leave the context at x^n
    return rc ? rc : rc2;
}

int ehd_evolve(ehd_ctx* ctx, const ehd_step_params* prm, double inv_pe, double t_end, double dt0, double tol,
               int max_steps, double* gamma_d, ehd_evolve_stats* stats)
{
    if (!ctx) return EHD_E_ARG;
    if (!ehd_ctx_ndrops(ctx)) return ehd_ctx_fail(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!gamma_d || !stats) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL argument");
    int rc = check_params(ctx, prm, inv_pe);
    if (rc) return rc;
    if (!(t_end >= 0.0) || !(dt0 > 0.0) || !(tol > 0.0) || max_steps < 1)
        return ehd_ctx_fail(ctx, EHD_E_ARG, "need t_end >= 0, dt0 > 0, tol > 0 and max_steps >= 1");
    EVO_HIP(hipSetDevice(ehd_ctx_device(ctx)));
    hipStream_t st = ehd_ctx_stream(ctx);
    Work w;
    if ((rc = make_work(ctx, w))) return rc;
    Buf xnew, gnew;
    if ((rc = alloc(ctx, xnew, 3 * w.nc)) || (rc = alloc(ctx, gnew, w.nc))) return rc;
    if ((rc = ehd_drop_coefs(ctx, w.xn.p))) return rc;
    stats->t = 0.0;
    stats->accepted = stats->rejected = 0;
    stats->matvecs = 0;
    stats->max_err = 0.0;
    double dt = dt0;
    ehd_step_report rep{};
    if ((rc = stage_a(ctx, w, prm, inv_pe, gamma_d, rep.iters))) return rc;
    stats->matvecs += rep.iters[0] + rep.iters[1];
    int steps = 0;
    while (stats->t < t_end * (1.0 - 1e-14) && steps < max_steps) {
        ++steps;
        const double h = std::min(dt, t_end - stats->t);
        if ((rc = step_b(ctx, w, prm, inv_pe, h, gamma_d, xnew.p, gnew.p, &rep))) return rc;
        stats->matvecs += rep.iters[2] + rep.iters[3] + rep.iters_gamma;
        const double err = std::max(rep.err_drop, rep.err_surf);
        if (err < tol) {                                      // accept
            stats->t += h;
            ++stats->accepted;
            stats->max_err = std::max(stats->max_err, err);
            EVO_HIP(hipMemcpyAsync(w.xn.p, xnew.p, sizeof(double) * 3 * w.nc, hipMemcpyDeviceToDevice, st));
            EVO_HIP(hipMemcpyAsync(gamma_d, gnew.p, sizeof(double) * w.nc, hipMemcpyDeviceToDevice, st));
            if ((rc = ehd_update_shape(ctx, w.xn.p))) return rc;
            // warm starts for the next first stage: the half-step solutions
            EVO_HIP(hipMemcpyAsync(w.enA.p, w.enB.p, sizeof(double) * w.nc, hipMemcpyDeviceToDevice, st));
            EVO_HIP(hipMemcpyAsync(w.uA.p, w.uB.p, sizeof(double) * 3 * w.nc, hipMemcpyDeviceToDevice, st));
            if ((rc = stage_a(ctx, w, prm, inv_pe, gamma_d, rep.iters))) return rc;
            stats->matvecs += rep.iters[0] + rep.iters[1];
        } else {                                              // reject: back to x^n, first stage still valid
            ++stats->rejected;
            if ((rc = ehd_update_shape(ctx, w.xn.p))) return rc;
        }
        // dt (0.9 tol / err)^(1/2), the growth bounded by 5 and the cut by 0.2
        const double fac = err > 0.0 ? std::sqrt(0.9 * tol / err) : 5.0;
        dt = h * std::min(5.0, std::max(0.2, fac));
    }
    stats->dt = dt;
    EVO_HIP(hipStreamSynchronize(st));
    return EHD_OK;
}

}  // extern "C"
