// Galerkin solvers built on the layer-potential evaluation (paper Sec. 2,
// eq. galerkin_En and eq. BIM_galerkin): restarted GMRES in FP64 on the
// device, whose mat-vec is one ehd_layer_potentials call followed by the
// Galerkin projection ehd_analyze.  Orthogonalisation is classical
// Gram-Schmidt applied twice (CGS2), with the dot products of a step batched
// in one launch; the small Hessenberg least-squares problem (Givens
// rotations) lives on the host.
//
// The unknowns are packed SH coefficient vectors (the layout of
// include/ehdbim.h); the imaginary slots of the m = 0 coefficients are
// carried along and stay zero (the projection writes zeros there and the
// right-hand sides have zeros there).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "ctx_access.h"
#include "ehdbim.h"

// Workspace of the allocation-free E_n solve (ehd_solve_En_noalloc): 8 Mi
// doubles (64 MiB), one copy on every device the library runs on, held
// until the process ends.  In host code its name stands for no device
// address: kernels and copies get the address that hipGetSymbolAddress
// returns on the device (scratch_of_device).
static __device__ __align__(256) double scratch[8LL << 20];

namespace {

constexpr int kT = 256;

// out[i] = <V_i, w>, one block per vector, fixed summation order.
__global__ __launch_bounds__(kT) void k_dots(const double* __restrict__ V, long long ld, const double* __restrict__ w,
                                             long long n, double* __restrict__ out)
{
    const double* v = V + (long long)blockIdx.x * ld;
    double s = 0.0;
    for (long long t = threadIdx.x; t < n; t += kT) s = fma(v[t], w[t], s);
    __shared__ double sh[kT];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// w -= sum_{i<k} h[i] V_i
__global__ void k_subtract(double* __restrict__ w, const double* __restrict__ V, long long ld, int k,
                           const double* __restrict__ h, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double s = w[t];
    for (int i = 0; i < k; ++i) s = fma(-h[i], V[(long long)i * ld + t], s);
    w[t] = s;
}

__global__ void k_fill(double* __restrict__ y, double v, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = v;
}

// y = d * x (elementwise)
__global__ void k_mul(const double* __restrict__ d, const double* __restrict__ x, double* __restrict__ y, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = d[t] * x[t];
}

// y = x - k * y (elementwise k)
__global__ void k_xmky(const double* __restrict__ x, const double* __restrict__ k, double* __restrict__ y, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = x[t] - k[t] * y[t];
}

// y = a x + b y
__global__ void k_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y, long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = a * x[t] + b * y[t];
}

// g = E_inf(x0) . n0 with E_inf = -grad phi_inf,
// phi_inf = -(E_u z + E_q (z^2 - (x^2 + y^2) / 2))  (uniform + quadrupole)
__global__ void k_einf_dot_n(const double* __restrict__ x0, const double* __restrict__ n0, long long T, double Eu,
                             double Eq, double* __restrict__ g)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const double x = x0[t], y = x0[T + t], z = x0[2 * T + t];
    g[t] = -Eq * x * n0[t] - Eq * y * n0[T + t] + (Eu + 2.0 * Eq * z) * n0[2 * T + t];
}

// Degree n of the packed entry k (complex index k / 2 = n(n+1)/2 + m).
__device__ __forceinline__ int packed_degree(int k)
{
    const int c = k >> 1;
    int n = (int)((sqrt(8.0 * c + 1.0) - 1.0) * 0.5);
    while ((n + 1) * (n + 2) / 2 <= c) ++n;
    while (n * (n + 1) / 2 > c) --n;
    return n;
}

// Euclidean norm of the block's ne doubles at v (block reduction, fixed order).
__device__ double block_norm(const double* __restrict__ v, int ne)
{
    __shared__ double sh[kT];
    double s = 0.0;
    for (int k = threadIdx.x; k < ne; k += kT) s = fma(v[k], v[k], s);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sqrt(sh[0]);
    __syncthreads();
    return r;
}

// Initial guess of drop blockIdx.x (ne packed doubles from off[d]):
//   M^{-1} b + kappa |b| gain (y std + mean)        (y != NULL)
//   M^{-1} b                                          (y == NULL)
// with M = diag(1 + kappa n(n+1)) and y the network's (FP32) output.
__global__ __launch_bounds__(kT) void k_guess(const long long* __restrict__ off, const double* __restrict__ kappa,
                                              const double* __restrict__ b, const float* __restrict__ y, int ny,
                                              const double* __restrict__ ymean, const double* __restrict__ ystd,
                                              const double* __restrict__ gain, double* __restrict__ guess)
{
    const int d = blockIdx.x;
    const long long o = off[d];
    const int ne = (int)(off[d + 1] - o);
    const double kd = kappa[d];
    const double bn = y ? block_norm(b + o, ne) : 0.0;
    for (int k = threadIdx.x; k < ne; k += kT) {
        const int n = packed_degree(k);
        double g = b[o + k] / (1.0 + kd * n * (n + 1.0));
        if (y) g += kd * bn * gain[k] * ((double)y[(long long)d * ny + k] * ystd[k] + ymean[k]);
        guess[o + k] = g;
    }
}

// Network inputs of drop blockIdx.x (all drops of degree p, nc = (p+1)(p+2)):
// [x without its degree-0 terms (3 nc), b / |b| (nc), log10 kappa], each
// entry standardised, (v - mean) / std, and stored as FP32.
__global__ __launch_bounds__(kT) void k_features(int nc, const double* __restrict__ xcoef,
                                                 const double* __restrict__ kappa, const double* __restrict__ b,
                                                 const double* __restrict__ mean, const double* __restrict__ stdv,
                                                 float* __restrict__ feat)
{
    const int d = blockIdx.x, nf = 4 * nc + 1;
    const double* bd = b + (long long)d * nc;
    const double* xd = xcoef + (long long)d * 3 * nc;
    const double bn = block_norm(bd, nc);
    for (int k = threadIdx.x; k < nf; k += kT) {
        double v;
        if (k < 3 * nc) v = (k % nc) < 2 ? 0.0 : xd[k];     // degree 0 (translation) drops out
        else if (k < 4 * nc) v = bd[k - 3 * nc] / bn;
        else v = log10(kappa[d]);
        feat[(long long)d * nf + k] = (float)((v - mean[k]) / stdv[k]);
    }
}

unsigned nblocks(long long n) { return (unsigned)((n + kT - 1) / kT); }

// Interface force density of the velocity equation at the target nodes
// (Sec. 1: eq. interfacial_force, eq. el_force with the Maxwell stress in
// units where eps~ eps_0 = 1, and the density -(f / Ca_E - f^E) of
// eq. main_eq):
//   E_t  = (I - n n) E_inf(x) - grad_S S_L[q]        (tangential field)
//   f^E  = ((1 - Q/R^2) E_n^2 - (1 - Q) |E_t|^2) / 2 n + (1 - Q/R) E_n E_t
//   f    = 2 gamma H n - gamma'(Gamma) grad_S Gamma
// gamma: clean 1; linear 1 + beta (1 - Gamma); Langmuir
// (1 + beta ln(1 - x_s Gamma)) / (1 + beta ln(1 - x_s)) (scaled so that
// gamma(1) = 1).  Inputs [c][T]: x, n, gradq = grad_S S_L[q], gradG =
// grad_S Gamma; H, En, Gam [T] (Gam NULL: Gamma = 1).  Output ftot[3][T].
struct ForceParams {
    double R, Q, CaE, Eu, Eq, beta, xs;
    int eos;
};
__global__ void k_forces(const double* __restrict__ x, const double* __restrict__ n, const double* __restrict__ H,
                         const double* __restrict__ gradq, const double* __restrict__ gradG,
                         const double* __restrict__ En, const double* __restrict__ Gam, long long T, ForceParams fp,
                         double* __restrict__ ftot)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const double X = x[t], Y = x[T + t], Z = x[2 * T + t];
    const double nx = n[t], ny = n[T + t], nz = n[2 * T + t];
    // applied field E_inf = -grad phi_inf, phi_inf = -(E_u z + E_q (z^2 - (x^2 + y^2)/2))
    const double ex = -fp.Eq * X, ey = -fp.Eq * Y, ez = fp.Eu + 2.0 * fp.Eq * Z;
    const double en_inf = ex * nx + ey * ny + ez * nz;
    const double tx = ex - en_inf * nx - gradq[t], ty = ey - en_inf * ny - gradq[T + t],
                 tz = ez - en_inf * nz - gradq[2 * T + t];
    const double e = En[t], et2 = tx * tx + ty * ty + tz * tz;
    const double fn = 0.5 * ((1.0 - fp.Q / (fp.R * fp.R)) * e * e - (1.0 - fp.Q) * et2);
    const double ft = (1.0 - fp.Q / fp.R) * e;
    double g = 1.0, dg = 0.0;
    const double G = Gam ? Gam[t] : 1.0;
    if (fp.eos == EHD_EOS_LINEAR) {
        g = 1.0 + fp.beta * (1.0 - G);
        dg = -fp.beta;
    } else if (fp.eos == EHD_EOS_LANGMUIR) {
        const double norm = 1.0 / (1.0 + fp.beta * log(1.0 - fp.xs));
        g = (1.0 + fp.beta * log(1.0 - fp.xs * G)) * norm;
        dg = -fp.beta * fp.xs / (1.0 - fp.xs * G) * norm;
    }
    const double hn = 2.0 * g * H[t];
    const double inv = 1.0 / fp.CaE;
    const double gx = gradG ? gradG[t] : 0.0, gy = gradG ? gradG[T + t] : 0.0, gz = gradG ? gradG[2 * T + t] : 0.0;
    ftot[t] = fn * nx + ft * tx - inv * (hn * nx - dg * gx);
    ftot[T + t] = fn * ny + ft * ty - inv * (hn * ny - dg * gy);
    ftot[2 * T + t] = fn * nz + ft * tz - inv * (hn * nz - dg * gz);
}



struct DevBuf {
    double* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

#define SOLVE_HIP(call)                                                                              \
    do {                                                                                             \
        hipError_t _e = (call);                                                                      \
        if (_e != hipSuccess) {                                                                      \
            char _b[256];                                                                            \
            snprintf(_b, sizeof(_b), "%s failed: %s", #call, hipGetErrorString(_e));                 \
            return ehd_ctx_fail(ctx, EHD_E_HIP, _b);                                                 \
        }                                                                                            \
    } while (0)

using Op = std::function<int(const double* in, double* out)>;

// Workspace of one GMRES(m) solve of vectors of length n.  Device: the
// Krylov basis V [(m+1) n], w [n] and hd [2m+3] (the projections of the
// two Gram-Schmidt passes and |w|^2); host: the Hessenberg matrix
// H [(m+1) m], the Givens rotations cs, sn [m], g, h [m+1], y [m] and the
// projections' host copy hh [2m+3].
struct GmresWork {
    double *V, *w, *hd;
    double *H, *cs, *sn, *g, *h, *y, *hh;
};

// Restarted GMRES(m) for A x = b on device vectors of length n; x holds the
// initial guess on entry.  Converged when the true relative residual
// |b - A x| / |b| <= tol.  Every workspace entry is written before it is
// read.
template <class OpT>
int gmres_ws(ehd_ctx* ctx, long long n, const OpT& A, const double* b, double* x, int m, int maxit, double tol,
             const GmresWork& ws, int* iters, double* relres)
{
    hipStream_t st = ehd_ctx_stream(ctx);
    double* V = ws.V;
    double* w = ws.w;
    double* hd = ws.hd;
    double *H = ws.H, *cs = ws.cs, *sn = ws.sn, *g = ws.g, *h = ws.h, *y = ws.y, *hh = ws.hh;
    auto norm = [&](const double* vec, double* out) -> int {
        hipLaunchKernelGGL(k_dots, dim3(1), dim3(kT), 0, st, vec, n, vec, n, hd);
        SOLVE_HIP(hipGetLastError());
        SOLVE_HIP(hipMemcpyAsync(out, hd, sizeof(double), hipMemcpyDeviceToHost, st));
        SOLVE_HIP(hipStreamSynchronize(st));
        *out = std::sqrt(*out);
        return EHD_OK;
    };
    double bnorm;
    int rc = norm(b, &bnorm);
    if (rc) return rc;
    *iters = 0;
    if (bnorm == 0.0) {
        hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(kT), 0, st, x, 0.0, n);
        SOLVE_HIP(hipGetLastError());
        SOLVE_HIP(hipStreamSynchronize(st));
        *relres = 0.0;
        return EHD_OK;
    }
    for (;;) {
        // true residual r = b - A x, into V_0
        if ((rc = A(x, w))) return rc;
        SOLVE_HIP(hipMemcpyAsync(V, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(kT), 0, st, -1.0, w, 1.0, V, n);
        SOLVE_HIP(hipGetLastError());
        double beta;
        if ((rc = norm(V, &beta))) return rc;
        *relres = beta / bnorm;
        if (*relres <= tol || *iters >= maxit) return EHD_OK;
        hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(kT), 0, st, 0.0, V, 1.0 / beta, V, n);
        std::fill(g, g + m + 1, 0.0);
        g[0] = beta;
        int jl = -1;
        for (int j = 0; j < m; ++j) {
            if ((rc = A(V + (size_t)j * n, w))) return rc;
            ++*iters;
            // CGS2: two passes of h = V^T w, w -= V h, the projections kept
            // on the device; one copy to the host per step
            double* const hd2 = hd + (m + 1);
            hipLaunchKernelGGL(k_dots, dim3(j + 1), dim3(kT), 0, st, V, n, w, n, hd);
            hipLaunchKernelGGL(k_subtract, dim3(nblocks(n)), dim3(kT), 0, st, w, V, n, j + 1, hd, n);
            hipLaunchKernelGGL(k_dots, dim3(j + 1), dim3(kT), 0, st, V, n, w, n, hd2);
            hipLaunchKernelGGL(k_subtract, dim3(nblocks(n)), dim3(kT), 0, st, w, V, n, j + 1, hd2, n);
            hipLaunchKernelGGL(k_dots, dim3(1), dim3(kT), 0, st, w, n, w, n, hd + 2 * m + 2);
            SOLVE_HIP(hipGetLastError());
            SOLVE_HIP(hipMemcpyAsync(hh, hd, sizeof(double) * (size_t)(2 * m + 3), hipMemcpyDeviceToHost, st));
            SOLVE_HIP(hipStreamSynchronize(st));
            const double hn = std::sqrt(hh[2 * m + 2]);
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i] + hh[m + 1 + i];
            H[(size_t)(j + 1) * m + j] = hn;
            // previous Givens rotations, then a new one zeroing H[j+1][j]
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            const double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
            const double rr = std::hypot(a, c);
            cs[j] = rr > 0.0 ? a / rr : 1.0;
            sn[j] = rr > 0.0 ? c / rr : 0.0;
            H[(size_t)j * m + j] = rr;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            jl = j;
            if (hn > 0.0) {
                hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(kT), 0, st, 1.0 / hn, w, 0.0, V + (size_t)(j + 1) * n,
                                   n);
                SOLVE_HIP(hipGetLastError());
            }
            if (std::fabs(g[j + 1]) / bnorm <= tol || *iters >= maxit || hn == 0.0) break;
        }
        // y = H^{-1} g (upper triangular), x += V y
        for (int i = jl; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k <= jl; ++k) s -= H[(size_t)i * m + k] * y[k];
            y[i] = s / H[(size_t)i * m + i];
        }
        for (int i = 0; i <= jl; ++i) h[i] = -y[i];
        SOLVE_HIP(hipMemcpyAsync(hd, h, sizeof(double) * (jl + 1), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_subtract, dim3(nblocks(n)), dim3(kT), 0, st, x, V, n, jl + 1, hd, n);
        SOLVE_HIP(hipGetLastError());
    }
}

// GMRES(m) with its workspace allocated for the call.
int gmres(ehd_ctx* ctx, long long n, const Op& A, const double* b, double* x, int m, int maxit, double tol,
          int* iters, double* relres)
{
    DevBuf Vb, wb, hb;
    SOLVE_HIP(hipMalloc(&Vb.p, sizeof(double) * (size_t)(m + 1) * n));
    SOLVE_HIP(hipMalloc(&wb.p, sizeof(double) * (size_t)n));
    // hd: first-pass projections [0, m], second-pass [m + 1, 2m + 1], |w|^2 at 2m + 2
    SOLVE_HIP(hipMalloc(&hb.p, sizeof(double) * (size_t)(2 * m + 3)));
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), h(m + 1), y(m), hh(2 * m + 3);
    const GmresWork ws{Vb.p, wb.p, hb.p, H.data(), cs.data(), sn.data(), g.data(), h.data(), y.data(), hh.data()};
    return gmres_ws(ctx, n, A, b, x, m, maxit, tol, ws, iters, relres);
}

int check_opts(ehd_ctx* ctx, int far_prec, int restart, int maxit, double tol)
{
    if (far_prec != EHD_FAR_FP64 && far_prec != EHD_FAR_FP32C)
        return ehd_ctx_fail(ctx, EHD_E_ARG, "invalid far_prec");
    if (restart < 1 || restart > 200) return ehd_ctx_fail(ctx, EHD_E_ARG, "restart must be in [1, 200]");
    if (maxit < 0) return ehd_ctx_fail(ctx, EHD_E_ARG, "maxit must be >= 0");
    if (!(tol > 0.0)) return ehd_ctx_fail(ctx, EHD_E_ARG, "tol must be > 0");
    return EHD_OK;
}

int check_En(ehd_ctx* ctx, double R, double Eu, double Eq, int far_prec, int restart, int maxit, double tol,
             const double* en_coef_d, const int* iters, const double* relres)
{
    if (!ctx) return EHD_E_ARG;
    if (!ehd_ctx_ndrops(ctx)) return ehd_ctx_fail(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!en_coef_d || !iters || !relres) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL argument");
    if (!(R > 0.0) || !std::isfinite(Eu) || !std::isfinite(Eq))
        return ehd_ctx_fail(ctx, EHD_E_ARG, "R must be > 0 and E_u, E_q finite");
    return check_opts(ctx, far_prec, restart, maxit, tol);
}

// The E_n system of eq. galerkin_En with device buffers grid [T], rhs [n],
// geo [6 T] and the GMRES workspace ws (NULL: GMRES allocates its own).
int solve_En_impl(ehd_ctx* ctx, double R, double Eu, double Eq, int far_prec, int restart, int maxit, double tol,
                  double* en_coef_d, int* iters, double* relres, double* grid, double* rhs, double* geo,
                  const GmresWork* ws)
{
    long long T, n;
    int rc;
    if ((rc = ehd_num_targets(ctx, &T)) || (rc = ehd_num_coefs(ctx, &n))) return rc;
    hipStream_t st = ehd_ctx_stream(ctx);
    // right-hand side R/(R+1) P[E_inf . n]
    if ((rc = ehd_target_geometry(ctx, geo, geo + 3 * T))) return rc;
    hipLaunchKernelGGL(k_einf_dot_n, dim3(nblocks(T)), dim3(kT), 0, st, geo, geo + 3 * T, T, Eu, Eq, grid);
    SOLVE_HIP(hipGetLastError());
    if ((rc = ehd_analyze(ctx, 1, grid, rhs))) return rc;
    hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(kT), 0, st, 0.0, rhs, R / (R + 1.0), rhs, n);
    SOLVE_HIP(hipGetLastError());
    // operator E -> E/2 - (R-1)/(R+1) P[K*[E]]
    const double c = (R - 1.0) / (R + 1.0);
    auto A = [&](const double* in, double* out) -> int {
        int r = ehd_layer_potentials(ctx, nullptr, nullptr, in, EHD_LAP_DLADJ, far_prec, grid, nullptr);
        if (!r) r = ehd_analyze(ctx, 1, grid, out);
        if (r) return r;
        hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(kT), 0, st, 0.5, in, -c, out, n);
        SOLVE_HIP(hipGetLastError());
        return EHD_OK;
    };
    if (ws) return gmres_ws(ctx, n, A, rhs, en_coef_d, restart, maxit, tol, *ws, iters, relres);
    return gmres(ctx, n, Op(A), rhs, en_coef_d, restart, maxit, tol, iters, relres);
}

// Allocation-free E_n solve: its workspace lives in `scratch`, one array per
// device (the address of the device's copy is looked up once per device,
// with that device current, and kept).
constexpr long long kNoAllocDoubles = 8LL << 20;   // 64 MiB
constexpr int kNoAllocMaxRestart = 64;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

static_assert(kNoAllocDoubles == (long long)(sizeof(scratch) / sizeof(double)), "scratch size");

// Device address of `scratch` on device `dev` (current): looked up on the
// first call on that device, then kept.
int scratch_of_device(ehd_ctx* ctx, int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return ehd_ctx_fail(ctx, EHD_E_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char b[200];
            snprintf(b, sizeof(b), "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                     hipGetErrorString(e));
            return ehd_ctx_fail(ctx, EHD_E_HIP, b);
        }
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return EHD_OK;
}

}  // namespace

extern "C" {

int ehd_solve_En(ehd_ctx* ctx, double R, double Eu, double Eq, int far_prec, int restart, int maxit, double tol,
                 double* en_coef_d, int* iters, double* relres)
{
    int rc = check_En(ctx, R, Eu, Eq, far_prec, restart, maxit, tol, en_coef_d, iters, relres);
    if (rc) return rc;
    SOLVE_HIP(hipSetDevice(ehd_ctx_device(ctx)));
    long long T, n;
    if ((rc = ehd_num_targets(ctx, &T)) || (rc = ehd_num_coefs(ctx, &n))) return rc;
    DevBuf grid, rhs, geo;
    SOLVE_HIP(hipMalloc(&grid.p, sizeof(double) * (size_t)T));
    SOLVE_HIP(hipMalloc(&rhs.p, sizeof(double) * (size_t)n));
    SOLVE_HIP(hipMalloc(&geo.p, sizeof(double) * (size_t)6 * T));
    return solve_En_impl(ctx, R, Eu, Eq, far_prec, restart, maxit, tol, en_coef_d, iters, relres, grid.p, rhs.p,
                         geo.p, nullptr);
}

int ehd_solve_En_noalloc(ehd_ctx* ctx, double R, double Eu, double Eq, int far_prec, int restart, int maxit,
                         double tol, double* en_coef_d, int* iters, double* relres)
{
    int rc = check_En(ctx, R, Eu, Eq, far_prec, restart, maxit, tol, en_coef_d, iters, relres);
    if (rc) return rc;
    if (restart > kNoAllocMaxRestart) {
        char b[128];
        snprintf(b, sizeof(b), "restart %d exceeds the allocation-free solve's maximum %d", restart,
                 kNoAllocMaxRestart);
        return ehd_ctx_fail(ctx, EHD_E_SHAPE, b);
    }
    if (ehd_ctx_graph_on(ctx))
        return ehd_ctx_fail(ctx, EHD_E_STATE, "graph mode records graphs (which allocates): switch it off first");
    const int dev = ehd_ctx_device(ctx);
    SOLVE_HIP(hipSetDevice(dev));
    long long T, n;
    if ((rc = ehd_num_targets(ctx, &T)) || (rc = ehd_num_coefs(ctx, &n))) return rc;
    const long long m = restart;
    // scratch layout (each piece 256-byte aligned): V, w, hd, grid, rhs, geo
    const long long sizes[6] = {(m + 1) * n, n, 2 * m + 3, T, n, 6 * T};
    long long offs[6], need = 0;
    for (int i = 0; i < 6; ++i) {
        offs[i] = need;
        need += (sizes[i] + 31) / 32 * 32;
    }
    if (need > kNoAllocDoubles) {
        char b[200];
        snprintf(b, sizeof(b),
                 "workspace of %lld doubles ((restart + 4) n + 7 T + ...) exceeds the allocation-free solve's "
                 "%lld (n = %lld coefficients, T = %lld targets)",
                 need, kNoAllocDoubles, n, T);
        return ehd_ctx_fail(ctx, EHD_E_SHAPE, b);
    }
    double* base = nullptr;
    if ((rc = scratch_of_device(ctx, dev, &base))) return rc;
    double H[(kNoAllocMaxRestart + 1) * kNoAllocMaxRestart], cs[kNoAllocMaxRestart], sn[kNoAllocMaxRestart],
        g[kNoAllocMaxRestart + 1], h[kNoAllocMaxRestart + 1], y[kNoAllocMaxRestart], hh[2 * kNoAllocMaxRestart + 3];
    const GmresWork ws{base + offs[0], base + offs[1], base + offs[2], H, cs, sn, g, h, y, hh};
    return solve_En_impl(ctx, R, Eu, Eq, far_prec, restart, maxit, tol, en_coef_d, iters, relres, base + offs[3],
                         base + offs[4], base + offs[5], &ws);
}

int ehd_solve_velocity(ehd_ctx* ctx, double lambda, const double* fcoef_d, int far_prec, int restart, int maxit,
                       double tol, double* ucoef_d, int* iters, double* relres)
{
    if (!ctx) return EHD_E_ARG;
    if (!ehd_ctx_ndrops(ctx)) return ehd_ctx_fail(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!fcoef_d || !ucoef_d || !iters || !relres) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL argument");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return ehd_ctx_fail(ctx, EHD_E_ARG, "lambda must be >= 0");
    int rc = check_opts(ctx, far_prec, restart, maxit, tol);
    if (rc) return rc;
    SOLVE_HIP(hipSetDevice(ehd_ctx_device(ctx)));
    long long T, nc;
    if ((rc = ehd_num_targets(ctx, &T)) || (rc = ehd_num_coefs(ctx, &nc))) return rc;
    const long long n = 3 * nc;
    hipStream_t st = ehd_ctx_stream(ctx);
    DevBuf grid, rhs;
    SOLVE_HIP(hipMalloc(&grid.p, sizeof(double) * (size_t)3 * T));
    SOLVE_HIP(hipMalloc(&rhs.p, sizeof(double) * (size_t)n));
    // right-hand side P[S[f]]
    if ((rc = ehd_layer_potentials(ctx, fcoef_d, nullptr, nullptr, EHD_STOKES_SL, far_prec, grid.p, nullptr))) return rc;
    if ((rc = ehd_analyze(ctx, 3, grid.p, rhs.p))) return rc;
    // operator u -> (lambda+1) u - (lambda-1) P[D[u]]
    const Op A = [&](const double* in, double* out) -> int {
        int r = ehd_layer_potentials(ctx, nullptr, in, nullptr, EHD_STOKES_DL, far_prec, grid.p, nullptr);
        if (!r) r = ehd_analyze(ctx, 3, grid.p, out);
        if (r) return r;
        hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(kT), 0, st, lambda + 1.0, in, -(lambda - 1.0), out, n);
        SOLVE_HIP(hipGetLastError());
        return EHD_OK;
    };
    return gmres(ctx, n, A, rhs.p, ucoef_d, restart, maxit, tol, iters, relres);
}

int ehd_explicit_step(ehd_ctx* ctx, const ehd_step_params* prm, const double* gamma_coef_d, double* en_coef_d,
                      double* ucoef_d, double* xnew_coef_d, int* iters)
{
    if (!ctx) return EHD_E_ARG;
    if (!ehd_ctx_ndrops(ctx)) return ehd_ctx_fail(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!prm || !en_coef_d || !ucoef_d || !xnew_coef_d) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL argument");
    if (!(prm->CaE > 0.0) || !(prm->R > 0.0) || !std::isfinite(prm->dt) || !std::isfinite(prm->Q))
        return ehd_ctx_fail(ctx, EHD_E_ARG, "CaE and R must be > 0, Q and dt finite");
    if (prm->eos != EHD_EOS_CLEAN && prm->eos != EHD_EOS_LINEAR && prm->eos != EHD_EOS_LANGMUIR)
        return ehd_ctx_fail(ctx, EHD_E_ARG, "invalid eos");
    if (prm->eos == EHD_EOS_LANGMUIR && !(prm->xs >= 0.0 && prm->xs < 1.0))
        return ehd_ctx_fail(ctx, EHD_E_ARG, "Langmuir coverage x_s must be in [0, 1)");
    int rc;
    int it_en = 0, it_u = 0;
    double rr;
    // i. E_n
    if ((rc = ehd_solve_En(ctx, prm->R, prm->Eu, prm->Eq, prm->far_prec, prm->restart, prm->maxit, prm->tol,
                           en_coef_d, &it_en, &rr)))
        return rc;
    long long T, nc;
    if ((rc = ehd_num_targets(ctx, &T)) || (rc = ehd_num_coefs(ctx, &nc))) return rc;
    hipStream_t st = ehd_ctx_stream(ctx);
    DevBuf q, val, geo, H, gq, gG, En, Gm, ft, fc;
    SOLVE_HIP(hipMalloc(&q.p, sizeof(double) * (size_t)nc));
    SOLVE_HIP(hipMalloc(&val.p, sizeof(double) * (size_t)T));
    SOLVE_HIP(hipMalloc(&geo.p, sizeof(double) * (size_t)6 * T));
    SOLVE_HIP(hipMalloc(&H.p, sizeof(double) * (size_t)T));
    SOLVE_HIP(hipMalloc(&gq.p, sizeof(double) * (size_t)3 * T));
    SOLVE_HIP(hipMalloc(&En.p, sizeof(double) * (size_t)T));
    SOLVE_HIP(hipMalloc(&ft.p, sizeof(double) * (size_t)3 * T));
    SOLVE_HIP(hipMalloc(&fc.p, sizeof(double) * (size_t)3 * nc));
    // ii-iii. tangential field: the surface potential phi_inf + S_L[q],
    // q = [[E_n]] = (1 - 1/R) E_n, projected; its surface gradient
    hipLaunchKernelGGL(k_axpby, dim3(nblocks(nc)), dim3(kT), 0, st, 1.0 - 1.0 / prm->R, en_coef_d, 0.0, q.p, nc);
    SOLVE_HIP(hipGetLastError());
    if ((rc = ehd_layer_potentials(ctx, nullptr, nullptr, q.p, EHD_LAP_SL, prm->far_prec, val.p, nullptr))) return rc;
    if ((rc = ehd_analyze(ctx, 1, val.p, q.p))) return rc;
    if ((rc = ehd_surface(ctx, 1, q.p, H.p, gq.p, nullptr))) return rc;
    if ((rc = ehd_target_geometry(ctx, geo.p, geo.p + 3 * T))) return rc;
    if ((rc = ehd_synthesize(ctx, 1, en_coef_d, En.p))) return rc;
    const double* gG_ptr = nullptr;
    const double* Gm_ptr = nullptr;
    if (gamma_coef_d && prm->eos != EHD_EOS_CLEAN) {
        SOLVE_HIP(hipMalloc(&gG.p, sizeof(double) * (size_t)3 * T));
        SOLVE_HIP(hipMalloc(&Gm.p, sizeof(double) * (size_t)T));
        if ((rc = ehd_surface(ctx, 1, gamma_coef_d, H.p, gG.p, nullptr))) return rc;
        if ((rc = ehd_synthesize(ctx, 1, gamma_coef_d, Gm.p))) return rc;
        gG_ptr = gG.p;
        Gm_ptr = Gm.p;
    }
    // iv-v. forces at the nodes, projected
    ForceParams fp{prm->R, prm->Q, prm->CaE, prm->Eu, prm->Eq, prm->beta, prm->xs, prm->eos};
    hipLaunchKernelGGL(k_forces, dim3(nblocks(T)), dim3(kT), 0, st, geo.p, geo.p + 3 * T, H.p, gq.p, gG_ptr, En.p,
                       Gm_ptr, T, fp, ft.p);
    SOLVE_HIP(hipGetLastError());
    if ((rc = ehd_analyze(ctx, 3, ft.p, fc.p))) return rc;
    // vi. velocity
    if ((rc = ehd_solve_velocity(ctx, prm->lambda, fc.p, prm->far_prec, prm->restart, prm->maxit, prm->tol, ucoef_d,
                                 &it_u, &rr)))
        return rc;
    // vii. x + dt u
    if ((rc = ehd_drop_coefs(ctx, xnew_coef_d))) return rc;
    hipLaunchKernelGGL(k_axpby, dim3(nblocks(3 * nc)), dim3(kT), 0, st, prm->dt, ucoef_d, 1.0, xnew_coef_d, 3 * nc);
    SOLVE_HIP(hipGetLastError());
    SOLVE_HIP(hipStreamSynchronize(st));
    if (iters) {
        iters[0] = it_en;
        iters[1] = it_u;
    }
    return EHD_OK;
}

int ehd_solve_surfactant(ehd_ctx* ctx, const double* kappa_h, const double* rhs_d, int precond, int restart,
                         int maxit, double tol, double* gamma_d, int* iters, double* relres)
{
    if (!ctx) return EHD_E_ARG;
    if (!ehd_ctx_ndrops(ctx)) return ehd_ctx_fail(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!kappa_h || !rhs_d || !gamma_d || !iters || !relres) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL argument");
    for (int d = 0; d < ehd_ctx_ndrops(ctx); ++d)
        if (!(kappa_h[d] >= 0.0) || !std::isfinite(kappa_h[d]))
            return ehd_ctx_fail(ctx, EHD_E_ARG, "kappa must be >= 0 for every drop");
    int rc = check_opts(ctx, EHD_FAR_FP64, restart, maxit, tol);
    if (rc) return rc;
    SOLVE_HIP(hipSetDevice(ehd_ctx_device(ctx)));
    long long T, n;
    if ((rc = ehd_num_targets(ctx, &T)) || (rc = ehd_num_coefs(ctx, &n))) return rc;
    hipStream_t st = ehd_ctx_stream(ctx);
    // diagonal preconditioner on the packed layout: 1 / (1 + kappa n(n+1)),
    // the inverse of the operator on the unit sphere (Lap_S Y_nm = -n(n+1) Y_nm)
    std::vector<double> dinv((size_t)n, 1.0), dfwd((size_t)n, 1.0), kv((size_t)n);
    {
        size_t o = 0;
        for (int d = 0; d < ehd_ctx_ndrops(ctx); ++d) {
            const int p = ehd_ctx_drop_p(ctx, d);
            for (int nn = 0; nn <= p; ++nn)
                for (int m = 0; m <= nn; ++m)
                    for (int part = 0; part < 2; ++part, ++o) {
                        kv[o] = kappa_h[d];
                        if (precond) {
                            dfwd[o] = 1.0 + kappa_h[d] * nn * (nn + 1.0);
                            dinv[o] = 1.0 / dfwd[o];
                        }
                    }
        }
    }
    DevBuf lap, H, grad, proj, tmp, di, df, kd;
    SOLVE_HIP(hipMalloc(&lap.p, sizeof(double) * (size_t)T));
    SOLVE_HIP(hipMalloc(&H.p, sizeof(double) * (size_t)T));
    SOLVE_HIP(hipMalloc(&grad.p, sizeof(double) * (size_t)3 * T));
    SOLVE_HIP(hipMalloc(&proj.p, sizeof(double) * (size_t)n));
    SOLVE_HIP(hipMalloc(&tmp.p, sizeof(double) * (size_t)n));
    SOLVE_HIP(hipMalloc(&di.p, sizeof(double) * (size_t)n));
    SOLVE_HIP(hipMalloc(&df.p, sizeof(double) * (size_t)n));
    SOLVE_HIP(hipMalloc(&kd.p, sizeof(double) * (size_t)n));
    SOLVE_HIP(hipMemcpyAsync(kd.p, kv.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    SOLVE_HIP(hipMemcpyAsync(di.p, dinv.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    SOLVE_HIP(hipMemcpyAsync(df.p, dfwd.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    // operator c -> c - kappa P[Lap_S c], applied to M^{-1} y (right preconditioning)
    const Op A = [&](const double* in, double* out) -> int {
        hipLaunchKernelGGL(k_mul, dim3(nblocks(n)), dim3(kT), 0, st, di.p, in, tmp.p, n);
        int r = ehd_surface(ctx, 1, tmp.p, H.p, grad.p, lap.p);
        if (!r) r = ehd_analyze(ctx, 1, lap.p, out);
        if (r) return r;
        hipLaunchKernelGGL(k_xmky, dim3(nblocks(n)), dim3(kT), 0, st, tmp.p, kd.p, out, n);
        SOLVE_HIP(hipGetLastError());
        return EHD_OK;
    };
    // y0 = M c0, solve, c = M^{-1} y
    hipLaunchKernelGGL(k_mul, dim3(nblocks(n)), dim3(kT), 0, st, df.p, gamma_d, gamma_d, n);
    SOLVE_HIP(hipGetLastError());
    if ((rc = gmres(ctx, n, A, rhs_d, gamma_d, restart, maxit, tol, iters, relres))) return rc;
    hipLaunchKernelGGL(k_mul, dim3(nblocks(n)), dim3(kT), 0, st, di.p, gamma_d, gamma_d, n);
    SOLVE_HIP(hipGetLastError());
    SOLVE_HIP(hipStreamSynchronize(st));
    return EHD_OK;
}

int ehd_surfactant_guess(ehd_ctx* ctx, const double* kappa_h, const double* rhs_d, const float* y_d, int ny,
                         const double* ymean_d, const double* ystd_d, const double* gain_d, double* guess_d)
{
    if (!ctx) return EHD_E_ARG;
    const int nd = ehd_ctx_ndrops(ctx);
    if (!nd) return ehd_ctx_fail(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!kappa_h || !rhs_d || !guess_d) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL argument");
    if (y_d && (!ymean_d || !ystd_d || !gain_d)) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL network scaling");
    std::vector<long long> off((size_t)nd + 1, 0);
    std::vector<double> kv((size_t)nd);
    for (int d = 0; d < nd; ++d) {
        const int p = ehd_ctx_drop_p(ctx, d);
        if (!(kappa_h[d] >= 0.0) || !std::isfinite(kappa_h[d]))
            return ehd_ctx_fail(ctx, EHD_E_ARG, "kappa must be >= 0 for every drop");
        if (y_d && ny != (p + 1) * (p + 2))
            return ehd_ctx_fail(ctx, EHD_E_SHAPE, "ny must be (p+1)(p+2) for every drop");
        off[d + 1] = off[d] + (long long)(p + 1) * (p + 2);
        kv[d] = kappa_h[d];
    }
    SOLVE_HIP(hipSetDevice(ehd_ctx_device(ctx)));
    hipStream_t st = ehd_ctx_stream(ctx);
    DevBuf offb, kb;
    SOLVE_HIP(hipMalloc(&offb.p, sizeof(long long) * off.size()));
    SOLVE_HIP(hipMalloc(&kb.p, sizeof(double) * kv.size()));
    SOLVE_HIP(hipMemcpyAsync(offb.p, off.data(), sizeof(long long) * off.size(), hipMemcpyHostToDevice, st));
    SOLVE_HIP(hipMemcpyAsync(kb.p, kv.data(), sizeof(double) * kv.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_guess, dim3(nd), dim3(kT), 0, st, reinterpret_cast<const long long*>(offb.p), kb.p, rhs_d,
                       y_d, ny, ymean_d, ystd_d, gain_d, guess_d);
    SOLVE_HIP(hipGetLastError());
    SOLVE_HIP(hipStreamSynchronize(st));
    return EHD_OK;
}

int ehd_learned_features(ehd_ctx* ctx, const double* kappa_h, const double* rhs_d, const double* mean_d,
                         const double* std_d, float* feat_d)
{
    if (!ctx) return EHD_E_ARG;
    const int nd = ehd_ctx_ndrops(ctx);
    if (!nd) return ehd_ctx_fail(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!kappa_h || !rhs_d || !mean_d || !std_d || !feat_d) return ehd_ctx_fail(ctx, EHD_E_ARG, "NULL argument");
    const int p = ehd_ctx_drop_p(ctx, 0);
    for (int d = 0; d < nd; ++d) {
        if (ehd_ctx_drop_p(ctx, d) != p) return ehd_ctx_fail(ctx, EHD_E_SHAPE, "every drop must have the same p");
        if (!(kappa_h[d] > 0.0) || !std::isfinite(kappa_h[d]))
            return ehd_ctx_fail(ctx, EHD_E_ARG, "kappa must be > 0 for every drop");
    }
    const int nc = (p + 1) * (p + 2);
    SOLVE_HIP(hipSetDevice(ehd_ctx_device(ctx)));
    hipStream_t st = ehd_ctx_stream(ctx);
    DevBuf x, kb;
    SOLVE_HIP(hipMalloc(&x.p, sizeof(double) * (size_t)3 * nc * nd));
    SOLVE_HIP(hipMalloc(&kb.p, sizeof(double) * (size_t)nd));
    int rc = ehd_drop_coefs(ctx, x.p);
    if (rc) return rc;
    SOLVE_HIP(hipMemcpyAsync(kb.p, kappa_h, sizeof(double) * nd, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_features, dim3(nd), dim3(kT), 0, st, nc, x.p, kb.p, rhs_d, mean_d, std_d, feat_d);
    SOLVE_HIP(hipGetLastError());
    SOLVE_HIP(hipStreamSynchronize(st));
    return EHD_OK;
}

}  // extern "C"
