// MI355X (gfx950) layer-potential library: HIP kernels and the C ABI declared
// in include/ehdbim.h.  Paper: Sorgentone, Tornberg & Vlahovska,
// arXiv 1811.10270, Sec. 2 (spectral representation, Galerkin form, layer
// operators) and Sec. 2.1 (regular, singular quadrature).
//
// Pipeline of one evaluation (all on the context's stream):
//   k_synth (densities on the far grids) -> k_src_dens (weighted source
//   records, FP64 and FP32) -> k_self (rotation + rotated-grid synthesis +
//   singular reduction, FP64) -> k_far64 / k_far32 (direct sums over the
//   other drops) -> k_combine (scaling, component selection).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include "ehdbim.h"
#include "tables.h"
#include "ctx_access.h"

using ehd::ncoef;
using ehd::nlon_of;
using ehd::tri;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInv4Pi = 0.25 / kPi;
constexpr int kThreads = 256;
constexpr int kTile = 256;        // far-field sources per LDS tile
constexpr int kRec64 = 14;        // x(3) n(3) w(1) wf(3) wu(3) wsig(1)
constexpr int kNearMaxM = 12;     // nearly singular targets: most check points per line
constexpr int kNearSplit = 16;    // source chunks per pair in the check-point sums
constexpr int kRec32 = 13;        // x-c(3) n(3) wf(3) wu(3) wsig(1)
constexpr int kMaxChunks = 16;    // far field: largest number of source chunks

// ---------------------------------------------------------------------------
// Device-side descriptors
// ---------------------------------------------------------------------------
struct LegTab {                // degree-p expansions on a degree-Q grid
    const double* P;           // [Q+1][ncoef(p)]   Pbar_n^m(cos theta_i)
    const double* dP;          // [Q+1][ncoef(p)]   dPbar_n^m/dtheta
    const double* wq;          // [Q+1] (2 pi / nlon) * w_i^G
    const double* wsing;       // [Q+1] (2 pi / nlon) * w_i^G * 2 sin(theta_i/2) sum_{n<=Q} P_n
    const double* rsin;        // [Q+1] 1 / sin theta_i
    const double* cth;         // [Q+1] cos theta_i
    const double* trig;        // [nlon][p+1][2] cos(m phi_l), sin(m phi_l)
    const double* afrag;       // singular grids: MFMA A fragments of the quarter-period
                               // cos/sin tables: [row tile][k-step (EC ES OC OS)][lane]
    const double* lfrag;       // singular grids: MFMA A fragments of the Legendre sums,
                               // [latitude block][wave][k-step][lane]; rows 0-7 Pbar,
                               // 8-15 dPbar/dtheta at 8 latitudes
    int p, Q, nlon, pad;
};

struct WigTab {                // rotation blocks for each latitude of the p-grid
    const double* A;           // [p+1][wig_block(p)]
    const double* B;
    int p, pad;
};

struct DropInfo {
    int p, qs, qf, nlon_p, nlon_s, nlon_f;
    int leg_pp, leg_ps, leg_pf, wig;
    long long coff;            // per-field coefficient offset (doubles)
    long long toff;            // first target node
    long long soff;            // first far-field source slot (tile aligned)
    long long ns;              // real far-field source nodes
    double c[3];               // reference centre (mean position)
};

// Column-major index of the (n, m) triangle, n = m..p: column m starts at
// column_start(p, m) = m (p + 1) - m (m - 1) / 2.
__host__ __device__ inline int column_start(int p, int m) { return m * (p + 1) - m * (m - 1) / 2; }

__device__ __forceinline__ int tri_n(int idx)
{
    int n = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while ((n + 1) * (n + 2) / 2 <= idx) ++n;
    while (n * (n + 1) / 2 > idx) --n;
    return n;
}

// Pointers read from descriptor structs are generic to the compiler; the
// tables and coefficients live in device global memory, so say so and get
// global (not flat) loads, which do not hold up LDS traffic.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p)
{
    return (const __attribute__((address_space(1))) T*)p;
}

// 1/sqrt(x) in FP64.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    // hardware estimate (relative error ~5e-8), then one third-order step:
    // with e = 1 - x y^2, x^(-1/2) = y (1 - e)^(-1/2) = y (1 + e/2 + 3 e^2/8 + O(e^3));
    // measured on MI355X: within 1.2 ulp over [1e-4, 1e4]
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

// 2/sqrt(x) in FP64 with one Newton step from the hardware estimate y:
// y (3 - x y^2), relative error about 3 e^2 / 8 with e = 1 - x y^2 (a few
// 1e-15).  Twice the reciprocal square root spares the step's halving (three
// instructions instead of four); the far-field sums take the powers of two
// out once per tile.  For those sums, whose terms are far from any
// cancellation at that level.
__device__ __forceinline__ double rsqrt2_newton(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-(x * y), y, 3.0);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// A double moved between lanes by a DPP pattern (both halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes, valid in every lane: within each row of 16 by DPP
// (swaps within quads, then the half-row and row mirrors; vector ALU, no
// LDS), then the four row sums read from lanes 0, 16, 32, 48.
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    double r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, 16 * k);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 16 * k);
        r[k] = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
    }
    return (r[0] + r[1]) + (r[2] + r[3]);
}

// ---------------------------------------------------------------------------
// Synthesis of K packed fields on a grid (own p-grid or far q-grid), one
// block per (drop, latitude).  Legendre sums per m into LDS, then the
// longitude sums per node.  Optional theta derivative and (1/sin) phi
// derivative (paper Sec. 2: derivatives from the SH coefficients).
// out[v * vstride + node], v = f (value), K+f (d/dtheta), 2K+f ((1/s) d/dphi).
// ---------------------------------------------------------------------------
template <int K, bool DERIV>
__global__ __launch_bounds__(kThreads) void k_synth(const DropInfo* __restrict__ drops,
                                                    const LegTab* __restrict__ legs, int far_grid,
                                                    const int2* __restrict__ rows,
                                                    const double* __restrict__ coef,
                                                    double* __restrict__ out, long long vstride)
{
    __shared__ double2 G[K][EHD_MAX_P + 1];
    __shared__ double2 Gd[DERIV ? K : 1][EHD_MAX_P + 1];
    const int2 r = rows[blockIdx.x];
    const DropInfo D = drops[r.x];
    const LegTab L = legs[far_grid ? D.leg_pf : D.leg_pp];
    const int p = L.p, i = r.y;
    const long nc = ncoef(p);
    const double* cf = coef + (long long)K * D.coff;
    const double* Prow = L.P + (long long)i * nc;
    const double* dProw = L.dP + (long long)i * nc;
    for (int it = threadIdx.x; it < K * (p + 1); it += blockDim.x) {
        const int f = it / (p + 1), m = it % (p + 1);
        double ar = 0.0, ai = 0.0, dr = 0.0, di = 0.0;
        for (int n = m; n <= p; ++n) {
            const long k = tri(n, m);
            const double cr = cf[2 * (f * nc + k)], ci = (m == 0) ? 0.0 : cf[2 * (f * nc + k) + 1];
            const double pv = Prow[k];
            ar += pv * cr;
            ai += pv * ci;
            if (DERIV) {
                const double dv = dProw[k];
                dr += dv * cr;
                di += dv * ci;
            }
        }
        G[f][m] = make_double2(ar, ai);
        if (DERIV) Gd[f][m] = make_double2(dr, di);
    }
    __syncthreads();
    const long long node0 = (far_grid ? D.soff : D.toff) + (long long)i * L.nlon;
    const double rs = L.rsin[i];
    for (int l = threadIdx.x; l < L.nlon; l += blockDim.x) {
        const double* tr = L.trig + (long long)l * (p + 1) * 2;
        double v[K], vt[K], vp[K];
        for (int f = 0; f < K; ++f) {
            v[f] = G[f][0].x;
            vt[f] = DERIV ? Gd[f][0].x : 0.0;
            vp[f] = 0.0;
        }
        for (int m = 1; m <= p; ++m) {
            const double c = tr[2 * m], s = tr[2 * m + 1];
            for (int f = 0; f < K; ++f) {
                const double2 g = G[f][m];
                v[f] += 2.0 * (g.x * c - g.y * s);
                if (DERIV) {
                    const double2 gd = Gd[f][m];
                    vt[f] += 2.0 * (gd.x * c - gd.y * s);
                    vp[f] -= 2.0 * m * (g.x * s + g.y * c);
                }
            }
        }
        for (int f = 0; f < K; ++f) {
            out[f * vstride + node0 + l] = v[f];
            if (DERIV) {
                out[(K + f) * vstride + node0 + l] = vt[f];
                out[(2 * K + f) * vstride + node0 + l] = vp[f] * rs;
            }
        }
    }
}

// Surface quantities at the target nodes (Sec. 1, eq. interfacial_force):
// mean curvature H = (1/2) div_S n and surface gradients of NG scalar fields.
// One block per (drop, latitude i) of the drop's own grid.  Per order m the
// partial sums over n of c Pbar, c dPbar/dtheta and c n(n+1) Pbar; the second
// theta-derivative follows from the associated Legendre equation,
//   d2Pbar/dtheta2 = -cot(theta) dPbar/dtheta - (n(n+1) - m^2/sin^2) Pbar.
// With x_t, x_p, x_tt, x_tp, x_pp the parameter derivatives of x, E F G and
// L M N the fundamental forms and W^2 = EG - F^2:
//   H = -(E N - 2 F M + G L) / (2 W^2),
//   grad_S g = ((G g_t - F g_p) x_t + (E g_p - F g_t) x_p) / W^2,
//   Lap_S g = (G h_tt - 2 F h_tp + E h_pp) / W^2,  h_ab = g_ab - x_ab . grad_S g
// (the trace of the surface Hessian).  Outputs H[T], grad[g][3][T] and, if
// lap is not NULL, lap[g][T].
template <int NG>
__global__ __launch_bounds__(kThreads) void k_surface(const DropInfo* __restrict__ drops,
                                                      const LegTab* __restrict__ legs,
                                                      const int2* __restrict__ rows,
                                                      const double* __restrict__ xcoef,
                                                      const double* __restrict__ gcoef, long long T,
                                                      double* __restrict__ Hout, double* __restrict__ grad,
                                                      double* __restrict__ lap)
{
    constexpr int K = 3 + NG;
    __shared__ double2 G0[K][EHD_MAX_P + 1], G1[K][EHD_MAX_P + 1], G2[K][EHD_MAX_P + 1];
    const int2 r = rows[blockIdx.x];
    const DropInfo D = drops[r.x];
    const LegTab L = legs[D.leg_pp];
    const int p = L.p, i = r.y;
    const long nc = ncoef(p);
    const double* Prow = L.P + (long long)i * nc;
    const double* dProw = L.dP + (long long)i * nc;
    for (int it = threadIdx.x; it < K * (p + 1); it += blockDim.x) {
        const int f = it / (p + 1), m = it % (p + 1);
        const double* cf = f < 3 ? xcoef + 3 * D.coff + f * 2 * nc : gcoef + (long long)NG * D.coff + (f - 3) * 2 * nc;
        double a0 = 0, b0 = 0, a1 = 0, b1 = 0, a2 = 0, b2 = 0;
        for (int n = m; n <= p; ++n) {
            const long k = tri(n, m);
            const double cr = cf[2 * k], ci = (m == 0) ? 0.0 : cf[2 * k + 1];
            const double pv = Prow[k], dv = dProw[k], nn = (double)n * (n + 1);
            a0 += pv * cr; b0 += pv * ci;
            a1 += dv * cr; b1 += dv * ci;
            a2 += nn * pv * cr; b2 += nn * pv * ci;
        }
        G0[f][m] = make_double2(a0, b0);
        G1[f][m] = make_double2(a1, b1);
        G2[f][m] = make_double2(a2, b2);
    }
    __syncthreads();
    const double rs = L.rsin[i];                           // 1 / sin theta
    const double ct = L.cth[i] * rs;                       // cot theta
    const long long node0 = D.toff + (long long)i * L.nlon;
    for (int l = threadIdx.x; l < L.nlon; l += blockDim.x) {
        const double* tr = L.trig + (long long)l * (p + 1) * 2;
        double vt[K], vp[K], vtt[K], vtp[K], vpp[K];
        for (int f = 0; f < K; ++f) {
            vt[f] = G1[f][0].x;
            vp[f] = 0.0;
            vtt[f] = -ct * G1[f][0].x - G2[f][0].x;
            vtp[f] = 0.0;
            vpp[f] = 0.0;
        }
        for (int m = 1; m <= p; ++m) {
            const double c = tr[2 * m], sn = tr[2 * m + 1], mm = (double)m * m * rs * rs;
            for (int f = 0; f < K; ++f) {
                const double2 g0 = G0[f][m], g1 = G1[f][m];
                vt[f] += 2.0 * (g1.x * c - g1.y * sn);
                vp[f] -= 2.0 * m * (g0.x * sn + g0.y * c);
                const double2 g2 = G2[f][m];
                const double er = -ct * g1.x - g2.x + mm * g0.x, ei = -ct * g1.y - g2.y + mm * g0.y;
                vtt[f] += 2.0 * (er * c - ei * sn);
                vtp[f] -= 2.0 * m * (g1.x * sn + g1.y * c);
                vpp[f] -= 2.0 * (double)m * m * (g0.x * c - g0.y * sn);
            }
        }
        const double E = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2];
        const double F = vt[0] * vp[0] + vt[1] * vp[1] + vt[2] * vp[2];
        const double Gg = vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2];
        double nx = vt[1] * vp[2] - vt[2] * vp[1], ny = vt[2] * vp[0] - vt[0] * vp[2], nz = vt[0] * vp[1] - vt[1] * vp[0];
        const double iw = rsqrt_nr(nx * nx + ny * ny + nz * nz);
        nx *= iw; ny *= iw; nz *= iw;
        const double Lf = vtt[0] * nx + vtt[1] * ny + vtt[2] * nz;
        const double Mf = vtp[0] * nx + vtp[1] * ny + vtp[2] * nz;
        const double Nf = vpp[0] * nx + vpp[1] * ny + vpp[2] * nz;
        const double iW2 = 1.0 / (E * Gg - F * F);
        const long long t = node0 + l;
        Hout[t] = -(E * Nf - 2.0 * F * Mf + Gg * Lf) * 0.5 * iW2;
        for (int g = 0; g < NG; ++g) {
            const double gt = vt[3 + g], gp = vp[3 + g];
            const double a = (Gg * gt - F * gp) * iW2, b = (E * gp - F * gt) * iW2;
            double htt = vtt[3 + g], htp = vtp[3 + g], hpp = vpp[3 + g];
            for (int c = 0; c < 3; ++c) {
                const double gr = a * vt[c] + b * vp[c];
                grad[((long long)g * 3 + c) * T + t] = gr;
                htt -= vtt[c] * gr;
                htp -= vtp[c] * gr;
                hpp -= vpp[c] * gr;
            }
            if (lap) lap[(long long)g * T + t] = (Gg * htt - 2.0 * F * htp + E * hpp) * iW2;
        }
    }
}

// Geometry from synthesized x, x_theta, x_phi/sin: n = x_t x x_ps / |.|,
// J = |x_t x x_ps|.  For targets: x0[3][T], n0[3][T].  For far sources:
// FP64 records x, n, w = (2 pi/nlon) w_i J, and the FP32 drop-centred copy.
__global__ void k_geom_targets(const double* __restrict__ syn, long long vstride, long long T,
                               double* __restrict__ x0, double* __restrict__ n0)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double xt[3], xp[3];
    for (int c = 0; c < 3; ++c) {
        x0[c * T + t] = syn[c * vstride + t];
        xt[c] = syn[(3 + c) * vstride + t];
        xp[c] = syn[(6 + c) * vstride + t];
    }
    const double cx = xt[1] * xp[2] - xt[2] * xp[1];
    const double cy = xt[2] * xp[0] - xt[0] * xp[2];
    const double cz = xt[0] * xp[1] - xt[1] * xp[0];
    const double ij = 1.0 / sqrt(cx * cx + cy * cy + cz * cz);
    n0[t] = cx * ij;
    n0[T + t] = cy * ij;
    n0[2 * T + t] = cz * ij;
}

// Area quadrature weights at the target nodes: w = (2 pi / nlon) w_j J, so
// that sum_t w[t] g[t] over a drop's nodes is the integral of g over its
// surface (eq. reg_quadrature).
__global__ void k_area_weights(const DropInfo* __restrict__ drops, const LegTab* __restrict__ legs,
                               const int* __restrict__ tdrop, const double* __restrict__ syn, long long vstride,
                               long long T, double* __restrict__ w)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const DropInfo D = drops[tdrop[t]];
    const int j = (int)((t - D.toff) / D.nlon_p);
    double xt[3], xp[3];
    for (int c = 0; c < 3; ++c) {
        xt[c] = syn[(3 + c) * vstride + t];
        xp[c] = syn[(6 + c) * vstride + t];
    }
    const double cx = xt[1] * xp[2] - xt[2] * xp[1];
    const double cy = xt[2] * xp[0] - xt[0] * xp[2];
    const double cz = xt[0] * xp[1] - xt[1] * xp[0];
    w[t] = legs[D.leg_pp].wq[j] * sqrt(cx * cx + cy * cy + cz * cz);
}

__global__ void k_geom_sources(const DropInfo* __restrict__ drops, const LegTab* __restrict__ legs,
                               const int* __restrict__ slot_drop, const double* __restrict__ syn,
                               long long vstride, long long Spad, double* __restrict__ src64,
                               float* __restrict__ src32)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Spad) return;
    const int d = slot_drop[s];
    const DropInfo D = drops[d];
    const long long local = s - D.soff;
    if (local >= D.ns) {  // padding slot: zero weight at the drop centre
        for (int c = 0; c < 3; ++c) {
            src64[c * Spad + s] = D.c[c];
            src64[(3 + c) * Spad + s] = 0.0;
            src32[c * Spad + s] = 0.0f;
            src32[(3 + c) * Spad + s] = 0.0f;
        }
        src64[6 * Spad + s] = 0.0;
        return;
    }
    const LegTab L = legs[D.leg_pf];
    const int i = (int)(local / L.nlon);
    double x[3], xt[3], xp[3];
    for (int c = 0; c < 3; ++c) {
        x[c] = syn[c * vstride + s];
        xt[c] = syn[(3 + c) * vstride + s];
        xp[c] = syn[(6 + c) * vstride + s];
    }
    const double cx = xt[1] * xp[2] - xt[2] * xp[1];
    const double cy = xt[2] * xp[0] - xt[0] * xp[2];
    const double cz = xt[0] * xp[1] - xt[1] * xp[0];
    const double J = sqrt(cx * cx + cy * cy + cz * cz);
    const double n[3] = {cx / J, cy / J, cz / J};
    for (int c = 0; c < 3; ++c) {
        src64[c * Spad + s] = x[c];
        src64[(3 + c) * Spad + s] = n[c];
        src32[c * Spad + s] = (float)(x[c] - D.c[c]);
        src32[(3 + c) * Spad + s] = (float)n[c];
    }
    src64[6 * Spad + s] = L.wq[i] * J;
}

// (2 rho_d)^2 of each drop, rho_d the largest distance of its far-grid
// nodes from its centre, into centre[4 d + 3]; one block per drop.
__global__ __launch_bounds__(kThreads) void k_drop_radius(const DropInfo* __restrict__ drops,
                                                          const double* __restrict__ src64, long long Spad,
                                                          double* __restrict__ centre)
{
    const DropInfo D = drops[blockIdx.x];
    double m = 0.0;
    for (long long s = D.soff + threadIdx.x; s < D.soff + D.ns; s += blockDim.x) {
        const double dx = src64[s] - D.c[0], dy = src64[Spad + s] - D.c[1], dz = src64[2 * Spad + s] - D.c[2];
        m = fmax(m, dx * dx + dy * dy + dz * dz);
    }
    __shared__ double red[kThreads];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) centre[4 * blockIdx.x + 3] = 4.0 * red[0];
}

// Weighted densities of the far-field sources (both precisions).
__global__ void k_src_dens(const double* __restrict__ synf, const double* __restrict__ synu,
                           const double* __restrict__ syns, long long vstride, long long Spad,
                           double* __restrict__ src64, float* __restrict__ src32)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Spad) return;
    const double w = src64[6 * Spad + s];
    for (int c = 0; c < 3; ++c) {
        const double f = synf ? w * synf[c * vstride + s] : 0.0;
        const double u = synu ? w * synu[c * vstride + s] : f;
        src64[(7 + c) * Spad + s] = f;
        src64[(10 + c) * Spad + s] = u;
        src32[(6 + c) * Spad + s] = (float)f;
        src32[(9 + c) * Spad + s] = (float)u;
    }
    const double sg = syns ? w * syns[s] : 0.0;
    src64[13 * Spad + s] = sg;
    src32[12 * Spad + s] = (float)sg;
}

// ---------------------------------------------------------------------------
// Singular self-interaction, one block per target (paper Sec. 2.1,
// eq. mod_weights and the rotation of the target to the north pole).
//   1. rotated coefficients c'_{nm'} = sum_m d^n_{m m'}(theta_t) e^{i m phi_t} c_nm
//      of every field, in the real form of tables.h, into LDS (vector ALU),
//      then into registers as the B operand of step 2a;
//   2. for each block of 8 latitudes t_i of the rotated degree-q grid:
//      a. Legendre sums G_f(m) = sum_n Pbar_n^m(t_i) c'_f(n,m) (and the theta
//         derivative table for x) as FP64 MFMA chains over the degrees n,
//         written as real Fourier coefficients (cos / sin of m phi) of every
//         grid quantity (x, x_theta, x_phi / sin theta, densities) into LDS;
//      b. longitude sums as FP64 MFMA products: the four nodes phi_l,
//         pi - phi_l, pi + phi_l and 2 pi - phi_l share the four partial
//         sums over (even m, odd m) x (cos, sin) terms, so four GEMMs of a
//         quarter of the rows and a quarter of the terms each, with the
//         cos/sin table as the register-resident A operand and the Fourier
//         coefficients as B (columns = grid quantities);
//      c. per node: normal, area factor, the kernels with the modified
//         weights, accumulated per thread;
//   3. block reduction.
// Fields in LDS: x(3) [f(3)] [u(3)] [sigma(1)]; D uses u when present, f
// otherwise.  Output: raw[comp][T] (already scaled by 1/(4 pi)).
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

// Longitude-sum geometry of the (p, q) rotated grid, N = nlon_q longitudes
// phi_l = 2 pi l / N, H = N / 2.  With the partial sums
//   EC = sum_{m even} a_m cos m phi, ES = sum_{m even} b_m sin m phi,
//   OC = sum_{m odd}  a_m cos m phi, OS = sum_{m odd}  b_m sin m phi,
// the nodes l, H - l, H + l, N - l take EC + ES + OC + OS, EC - ES - OC + OS,
// EC + ES - OC - OS and EC - ES + OC - OS (cos m(pi -+ phi) = (-1)^m cos m phi,
// sin m(pi - phi) = -(-1)^m sin m phi), so rows l = 0..floor(H/2) suffice.
// Row 0 (phi = 0 and pi) has no sine terms and all cosines 1: its values
// EC + OC and EC - OC are plain sums.  Where the degree class allows it
// (row0), row 0 is taken apart from the GEMM rows (which then start at
// l0 = 1) when that lowers the padded tile count.
//   nT row tiles of 16 (padded to nTp in {1, 2, 4, 8} so that the waves
//   split the tiles evenly); term counts: EC floor(p/2)+1 (m = 0, 2, ..),
//   ES floor(p/2) (m = 2, 4, ..), OC = OS = ceil(p/2) (m = 1, 3, ..);
//   k-steps of 4 terms per group, groups stored in the order EC ES OC OS.
struct QuarterGrid {
    int H, l0, rows, nT, nTp, nk[4], base[4], nks;
};
__host__ __device__ inline int padded_tiles(int nt) { return nt <= 1 ? 1 : nt <= 2 ? 2 : nt <= 4 ? 4 : 8; }
__host__ __device__ inline QuarterGrid quarter_grid(int p, int nlonq, bool row0)
{
    QuarterGrid g;
    g.H = nlonq / 2;
    const int with0 = padded_tiles((g.H / 2 + 1 + 15) / 16), without0 = padded_tiles((g.H / 2 + 15) / 16);
    g.l0 = (row0 && without0 < with0) ? 1 : 0;
    g.rows = g.H / 2 + 1 - g.l0;           // GEMM rows l = l0 .. floor(H/2)
    g.nT = (g.rows + 15) / 16;
    g.nTp = padded_tiles(g.nT);
    const int terms[4] = {p / 2 + 1, p / 2, (p + 1) / 2, (p + 1) / 2};
    int b = 0;
    for (int q = 0; q < 4; ++q) {
        g.nk[q] = (terms[q] + 3) / 4;
        g.base[q] = 4 * b;                 // first G row of the group
        b += g.nk[q];
    }
    g.nks = b;
    return g;
}

// Compile-time bounds of one degree class (all p <= PMAX; the rotated grid
// has at most 8 row tiles of 16 half-period longitudes).
constexpr int kLatBlock = 8;          // rotated latitudes per Legendre MFMA block

// Degree columns m = 0..p are dealt to the NW waves in snake order
// (0,1,..,NW-1, NW-1,..,0, 0,1,..); column m has ceil((p+1-m)/4) k-steps.
__host__ __device__ constexpr int snake_wave(int m, int nw)
{
    return ((m / nw) & 1) ? nw - 1 - (m % nw) : (m % nw);
}

constexpr int wave_ksteps_max(int PMAX, int nw)   // max over p <= PMAX and waves
{
    int best = 0;
    for (int p = 1; p <= PMAX; ++p)
        for (int w = 0; w < nw; ++w) {
            int t = 0;
            for (int m = 0; m <= p; ++m)
                if (snake_wave(m, nw) == w) t += (p + 1 - m + 3) / 4;
            best = t > best ? t : best;
        }
    return best;
}

// Slot of workgroup `bid` when the workgroups of a grid of `nb` are dealt to
// the kXcd XCDs round-robin and XCD x takes the contiguous slots
// [x q + min(x, r), ...), q = nb / kXcd, r = nb % kXcd (a bijection).
constexpr int kXcd = 8;
__device__ __forceinline__ unsigned xcd_slot(unsigned bid, unsigned nb)
{
    const unsigned q = nb / kXcd, r = nb % kXcd, x = bid % kXcd, pos = bid / kXcd;
    return x * q + (x < r ? x : r) + pos;
}

template <int PMAX>
struct SelfClass {
    static constexpr int KEC = (PMAX / 2 + 1 + 3) / 4;         // max k-steps per group
    static constexpr int KES = (PMAX / 2 + 3) / 4;
    static constexpr int KOC = ((PMAX + 1) / 2 + 3) / 4;
    static constexpr int NT = 512;                             // threads per block
    static constexpr int NW = NT / 64;                         // waves per block
    static constexpr int TPW = (8 + NW - 1) / NW;              // row tiles per wave (max)
    static constexpr int KW = wave_ksteps_max(PMAX, NW);       // Legendre k-steps per wave
    // row 0 of the longitude sums may be taken apart (pays at q = 2p for
    // p = 16 and 32: one tile less; elsewhere the tile count is unchanged)
    static constexpr bool ROW0 = PMAX == 16 || PMAX == 32;
    // rotation loop unroll (measured: 2 for p <= 24, 4 above)
    static constexpr int RU = PMAX <= 24 ? 2 : 4;
    // Legendre A fragments per prefetch batch: the default (measured best:
    // 5 for p <= 48, 3 for p <= 32, 2 below) and the two others built for the
    // field set x, f, sigma, among which the self-interaction autotuner picks
    static constexpr int PF = PMAX == 48 ? 5 : PMAX == 32 ? 3 : 2;
    static constexpr int PF_ALT0 = PMAX == 48 ? 3 : PMAX == 32 ? 2 : 3;
    static constexpr int PF_ALT1 = PMAX == 48 ? 6 : PMAX == 32 ? 5 : 4;
};

// Legendre k-steps per wave of the degree class of p (table stride per wave).
static inline int self_kw(int p)
{
    return p <= 16 ? SelfClass<16>::KW : p <= 24 ? SelfClass<24>::KW : p <= 32 ? SelfClass<32>::KW : SelfClass<48>::KW;
}
// Whether the degree class of p may take row 0 of the longitude sums apart.
static inline bool self_row0(int p)
{
    return p <= 16 ? SelfClass<16>::ROW0 : p <= 24 ? SelfClass<24>::ROW0 : p <= 32 ? SelfClass<32>::ROW0 : SelfClass<48>::ROW0;
}

template <int PMAX, bool HF, bool HU, bool HS, int PFT = 0>
__global__ __launch_bounds__(SelfClass<PMAX>::NT) void k_self(
    const DropInfo* __restrict__ drops, const LegTab* __restrict__ legs,
    const WigTab* __restrict__ wigs, const int* __restrict__ order, const int* __restrict__ tdrop,
    const double* __restrict__ xcoef, const double* __restrict__ fcoef,
    const double* __restrict__ ucoef, const double* __restrict__ scoef,
    const double* __restrict__ tx, const double* __restrict__ tnrm, long long T, unsigned kinds,
    double* __restrict__ raw)
{
    constexpr int NF = 3 + (HF ? 3 : 0) + (HU ? 3 : 0) + (HS ? 1 : 0);
    constexpr int FOFF = 3, UOFF = 3 + (HF ? 3 : 0), SOFF = 3 + (HF ? 3 : 0) + (HU ? 3 : 0);
    constexpr int NV = NF + 6;           // + x_theta(3), x_phi/sin(3)
    constexpr int VD = 9;                // first density variant
    using SC = SelfClass<PMAX>;
    static_assert(2 * NF <= 16, "at most 8 fields: (field, re/im) fill the 16 MFMA columns");
    static_assert(SC::NW == 8, "row tiles (up to 8) are split evenly over 8 waves");
    constexpr int NT = SC::NT, NW = SC::NW, LB = kLatBlock;
    extern __shared__ double2 lds[];
    __shared__ double red[NW][9];

    // Workgroups go to the 8 XCDs round-robin; give each XCD a contiguous
    // range of the cost-ordered target list, so that the blocks sharing an
    // L2 work on neighbouring targets (same rotation tables).
    const long long tg = order[xcd_slot(blockIdx.x, gridDim.x)];
    const int d = tdrop[tg];
    const DropInfo D = drops[d];
    const int p = D.p;
    const long nc = ncoef(p);
    const int node = (int)(tg - D.toff), j = node / D.nlon_p, k = node % D.nlon_p;
    const LegTab Lq = legs[D.leg_ps];
    const LegTab Lp = legs[D.leg_pp];
    const WigTab W = wigs[D.wig];
    const QuarterGrid qg = quarter_grid(p, Lq.nlon, SC::ROW0);
    double2* cr = lds;                               // [NF][nc] rotated coefficients
    double* R = reinterpret_cast<double*>(lds);      // later: Fourier blocks + node values
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    (void)NT;

    const __attribute__((address_space(1))) double* fld[NF];
    for (int c = 0; c < 3; ++c) fld[c] = gmem(xcoef + 3 * D.coff + c * 2 * nc);
    if constexpr (HF) for (int c = 0; c < 3; ++c) fld[FOFF + c] = gmem(fcoef + 3 * D.coff + c * 2 * nc);
    if constexpr (HU) for (int c = 0; c < 3; ++c) fld[UOFF + c] = gmem(ucoef + 3 * D.coff + c * 2 * nc);
    if constexpr (HS) fld[SOFF] = gmem(scoef + D.coff);

    // register-resident A operand of the longitude sums of this wave's row
    // tile (rows l = 16 tile .. 16 tile + 15): cos/sin(m phi_l) of the four
    // term groups.  Waves w, w + nTp, .. share tile w % nTp and split the
    // latitudes of a block.  Loaded here, before the rotation, whose time
    // hides their latency.
    const int my_tile = wv % qg.nTp;
    const bool dft_wave = my_tile < qg.nT;
    double aEC[SC::KEC], aES[SC::KES], aOC[SC::KOC], aOS[SC::KOC];
    {
        const auto src = gmem(Lq.afrag + (long long)(dft_wave ? my_tile : 0) * qg.nks * 64 + lane);
#pragma unroll
        for (int ks = 0; ks < SC::KEC; ++ks)
            aEC[ks] = (dft_wave && ks < qg.nk[0]) ? src[(long long)(qg.base[0] / 4 + ks) * 64] : 0.0;
#pragma unroll
        for (int ks = 0; ks < SC::KES; ++ks)
            aES[ks] = (dft_wave && ks < qg.nk[1]) ? src[(long long)(qg.base[1] / 4 + ks) * 64] : 0.0;
#pragma unroll
        for (int ks = 0; ks < SC::KOC; ++ks) {
            aOC[ks] = (dft_wave && ks < qg.nk[2]) ? src[(long long)(qg.base[2] / 4 + ks) * 64] : 0.0;
            aOS[ks] = (dft_wave && ks < qg.nk[3]) ? src[(long long)(qg.base[3] / 4 + ks) * 64] : 0.0;
        }
    }

    // 1. rotation, into LDS (column-major: column m holds n = m..p
    //    contiguously).
    //    a. z_nm = c_nm e^{i m phi_t} of every field, in the slots the rotated
    //       coefficients of degree n will take;
    //    b. each degree n belongs to one wave (snake order over the waves),
    //       lane m' computes Re c'_nm' = sum_m A_mm' Re z_nm and
    //       Im c'_nm' = sum_m B_mm' Im z_nm for all fields (z read as LDS
    //       broadcasts, the rows of A and B coalesced over the lanes), then
    //       overwrites the degree's slots: only this wave reads them.
    static_assert(PMAX < 64, "one lane per order m' of a degree");
    {
        const auto ph = gmem(Lp.trig + (long long)k * (p + 1) * 2);
        for (int it = threadIdx.x; it < nc; it += blockDim.x) {
            const int n = tri_n(it), m = it - n * (n + 1) / 2;
            const int cpos = column_start(p, m) + n - m;
            const double cm = ph[2 * m], sm = ph[2 * m + 1];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double c0 = fld[f][2 * it], c1 = m ? fld[f][2 * it + 1] : 0.0;
                cr[f * nc + cpos] = make_double2(c0 * cm - c1 * sm, c0 * sm + c1 * cm);
            }
        }
    }
    __syncthreads();
    {
        const long wb = ehd::wig_block(p);
        const auto A = gmem(W.A + (long long)j * wb);
        const auto B = gmem(W.B + (long long)j * wb);
        // Jobs: each degree >= 2 npair alone (64 lanes, m' = lane), then the
        // pairs (2k, 2k+1) of degrees <= 31 on the two half-waves (m' =
        // lane % 32), so that each LDS broadcast of z_nm serves two degrees
        // (the rotation is bound by those broadcasts).  Jobs by decreasing
        // length, dealt to the waves in snake order.
        const int npair = min(p + 1, 32) / 2, nsingle = p + 1 - 2 * npair, njob = nsingle + npair;
        const int dn0 = 2 * NW - 1 - 2 * wv, dn1 = 2 * wv + 1;
        bool odd = false;
        for (int J = wv; J < njob; J += odd ? dn1 : dn0, odd = !odd) {
            const bool single = J < nsingle;                               // wave-uniform
            const int k2 = single ? 0 : 2 * (npair - 1 - (J - nsingle));
            const int nmax = single ? p - J : k2 + 1;                      // last order m of the job
            const int n = single ? nmax : k2 + (lane >> 5);                // this lane's degree
            const int mpl = single ? lane : (lane & 31);                   // this lane's order m'
            const int mp = mpl <= n ? mpl : n;            // lanes past n repeat m' = n, store nothing
            const auto An = A + ehd::wig_off(n) + mp;
            const auto Bn = B + ehd::wig_off(n) + mp;
            double are[NF], aim[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) { are[f] = 0.0; aim[f] = 0.0; }
            const double2* zn = cr + column_start(p, 0) + n;   // z_n0 of field 0; z_nm at + column_start(p, m) - m
#pragma unroll SC::RU
            for (int m = 0; m <= nmax; ++m) {
                // the lower degree of a pair has no order m = nmax: weight 0 (its
                // z address then lies in the next column, in bounds)
                const bool on = m <= n;
                const int mm = on ? m : n;
                const double a = on ? An[mm * (n + 1)] : 0.0, b = on ? Bn[mm * (n + 1)] : 0.0;
                const int zo = column_start(p, m) - m;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const double2 z = zn[f * nc + zo];
                    are[f] = fma(a, z.x, are[f]);
                    aim[f] = fma(b, z.y, aim[f]);
                }
            }
            if (mpl <= n) {
                const int cpos = column_start(p, mpl) + n - mpl;
#pragma unroll
                for (int f = 0; f < NF; ++f) cr[f * nc + cpos] = make_double2(are[f], aim[f]);
            }
        }
    }
    __syncthreads();

    // 2. rotated coefficients into registers as the B operand of the Legendre
    //    MFMA: wave wv owns the degree columns m with snake_wave(m) == wv,
    //    walked in increasing m as one sequence of k-steps t; lane holds
    //    c'_f(n, m) (re or im) for column (f, re/im) = lane % 16 and
    //    n = m + 4 ks + lane / 16.
    double cB[SC::KW];
    const int ci = lane & 15, cf_ = ci >> 1, cri = ci & 1;
    {
        // this wave's columns in snake order: m = wv, then steps of dn0 and
        // dn1 in turn (wave-uniform, straight-line, so the loads issue together)
        const int dn0 = 2 * NW - 1 - 2 * wv, dn1 = 2 * wv + 1;
        int m = wv, ks = 0;
        bool odd = false;
        int left = (m <= p) ? (p + 1 - m + 3) / 4 : 0;
#pragma unroll
        for (int t = 0; t < SC::KW; ++t) {
            const int n = m + 4 * ks + (lane >> 4);
            const bool ok = left > 0 && cf_ < NF && n <= p;
            const int idx = ok ? cf_ * (int)nc + column_start(p, m) + n - m : 0;
            const double2 c = cr[idx];
            cB[t] = ok ? (cri ? c.y : c.x) : 0.0;
            if (left > 0) {
                --left;
                ++ks;
                if (left == 0) {
                    m += odd ? dn1 : dn0;
                    odd = !odd;
                    ks = 0;
                    left = (m <= p) ? (p + 1 - m + 3) / 4 : 0;
                }
            }
        }
    }
    __syncthreads();   // LDS free: Fourier blocks and per-wave node buffers from here on

    const int gsz = qg.nks * 64;                      // one latitude's Fourier block
    constexpr int NVP = NV | 1;                       // node record stride (odd: fewer bank conflicts)
    // node buffer per wave: 64 records (+ spare slots for the pipelined
    // stores of p <= 32)
    constexpr int NBW = 64 * NVP + (PMAX <= 32 ? 16 : 0);
    double* NB = R + LB * gsz + wv * NBW;             // this wave's node values (64 nodes)
    // Rows and columns of a Fourier block that are not rewritten meet zero A
    // entries (padding terms) or feed unused output columns; start from zeros.
    for (int z = threadIdx.x; z < LB * gsz; z += blockDim.x) R[z] = 0.0;
    __syncthreads();   // every zero is written before any wave stores Legendre sums there

    double x0[3], n0v[3];
    for (int c = 0; c < 3; ++c) { x0[c] = tx[c * T + tg]; n0v[c] = tnrm[c * T + tg]; }
    double acc[9];
    for (int c = 0; c < 9; ++c) acc[c] = 0.0;
    const bool wS = (kinds & EHD_STOKES_SL) && HF;
    const bool wD = (kinds & EHD_STOKES_DL) && (HF || HU);
    const bool wSL = (kinds & EHD_LAP_SL) && HS, wL = (kinds & EHD_LAP_DL) && HS;
    const bool wK = (kinds & EHD_LAP_DLADJ) && HS;
    const int nblk = (Lq.Q + 1 + LB - 1) / LB;
    const auto rsin = gmem(Lq.rsin);
    const auto wsing = gmem(Lq.wsing);

    // Legendre sums of degree m for the 8 latitudes of a block, from the MFMA
    // result (rows: Pbar at latitudes 0..7, then dPbar/dtheta at 0..7;
    // element r of the lane holds row lane/16 + 4 r, column (field, re/im)),
    // stored as real Fourier coefficients: field values and x_theta in the
    // cos row (re) or sin row (im) of m with factors 1 (m = 0) or 2 and -2,
    // x_phi / sin theta = -m (a_m sin - b_m cos) / sin theta in the other row.
    // Kept short: it is expanded at every k-step of the unrolled chain.
    const int f_l = cf_ < NF ? cf_ : 0;
    const int v_l = (f_l < 3) ? f_l : VD + (f_l - 3);
    const bool lane_xf = cf_ < 3, lane_field = cf_ < NF;
    double* const Gl0 = R + (lane >> 4) * gsz;          // this lane's latitudes 0..3 of the block
    double* const Gl1 = Gl0 + 4 * gsz;                  // and 4..7
    // alternating steps between the snake-ordered columns of this wave
    const int dm0 = 2 * NW - 1 - 2 * wv, dm1 = 2 * wv + 1;
    auto store_col = [&](int m, const dbl4& a, double rs0, double rs1) {
        if (!lane_field || (m == 0 && cri)) return;
        const int kc = (m & 1) ? qg.base[2] + (m - 1) / 2 : m / 2;
        const int ksr = (m & 1) ? qg.base[3] + (m - 1) / 2 : qg.base[1] + m / 2 - 1;
        const int r12 = (cri ? ksr : kc) * 16, r3 = (cri ? kc : ksr) * 16;
        const double sc = (m == 0) ? 1.0 : (cri ? -2.0 : 2.0);
        Gl0[r12 + v_l] = sc * a[0];
        Gl1[r12 + v_l] = sc * a[1];
        if (lane_xf) {
            Gl0[r12 + 3 + f_l] = sc * a[2];
            Gl1[r12 + 3 + f_l] = sc * a[3];
            if (m > 0) {
                const double sx = -2.0 * m;
                Gl0[r3 + 6 + f_l] = sx * rs0 * a[0];
                Gl1[r3 + 6 + f_l] = sx * rs1 * a[1];
            }
        }
    };

    const int m_first = wv <= p ? wv : p + 1;
    // Legendre fragments per prefetch batch (PFT, else the class default)
    constexpr int PF = PFT > 0 ? PFT : SC::PF;
    constexpr int NBATCH = (SC::KW + PF - 1) / PF;
    // kernels at one node (its NV values in val: this lane's record of the
    // wave's node buffer or of the row-0 records) with the modified weight wi of its
    // latitude (0 for a lane without a node of its own), accumulated per
    // lane.  gate: skip the kinds not requested (branches); without it
    // every kind the fields allow is accumulated (the requested ones are
    // stored) and the code has no branch, so the scheduler can interleave
    // it with the next latitude's longitude-sum MFMAs.
    auto eval_node = [&](const double* val, double wi, bool gate) {
        const double xt0 = val[3], xt1 = val[4], xt2 = val[5];
        const double xp0 = val[6], xp1 = val[7], xp2 = val[8];
        const double cx = xt1 * xp2 - xt2 * xp1;
        const double cy = xt2 * xp0 - xt0 * xp2;
        const double cz = xt0 * xp1 - xt1 * xp0;
        // ungated, lanes without a node (weight 0) may hold padding rows of
        // the longitude sums (zeros): keep their arithmetic finite (gated
        // calls come from lanes with a node only)
        const bool live = gate || wi != 0.0;
        const double J2 = live ? cx * cx + cy * cy + cz * cz : 1.0;
        const double iJ = rsqrt_nr(J2);
        const double w = wi * J2 * iJ;
        const double nx = cx * iJ, ny = cy * iJ, nz = cz * iJ;
        const double hx = x0[0] - val[0], hy = x0[1] - val[1], hz = x0[2] - val[2];
        const double r2 = live ? hx * hx + hy * hy + hz * hz : 1.0;
        const double ir = rsqrt_nr(r2), ir2 = ir * ir, ir3 = ir * ir2;
        const double hn = hx * nx + hy * ny + hz * nz;
        if constexpr (HF) {
            if (!gate || wS) {
                const double f0 = val[VD], f1 = val[VD + 1], f2 = val[VD + 2];
                const double hf = (hx * f0 + hy * f1 + hz * f2) * ir3;
                acc[0] += w * (f0 * ir + hx * hf);
                acc[1] += w * (f1 * ir + hy * hf);
                acc[2] += w * (f2 * ir + hz * hf);
            }
        }
        if constexpr (HF || HU) {
            if (!gate || wD) {
                constexpr int uo = VD + (HU ? UOFF : FOFF) - 3;
                const double hu = hx * val[uo] + hy * val[uo + 1] + hz * val[uo + 2];
                const double tq = -6.0 * w * hu * hn * ir3 * ir2;
                acc[3] += tq * hx;
                acc[4] += tq * hy;
                acc[5] += tq * hz;
            }
        }
        if constexpr (HS) {
            const double sg = w * val[VD + SOFF - 3];
            if (!gate || wSL) acc[6] += sg * ir;
            if (!gate || wL) acc[7] += sg * hn * ir3;
            if (!gate || wK) acc[8] += sg * (hx * n0v[0] + hy * n0v[1] + hz * n0v[2]) * ir3;
        }
    };

    // Row 0 of the longitude sums (when taken apart): each wave stores the two
    // nodes (phi = 0, pi) of its latitude in the block's row-0 records, and
    // after the block's last barrier one wave evaluates all sixteen in
    // sixteen lanes (during the next block's Legendre sums), instead of two
    // lanes in each of the eight waves.
    double* const RZ = R + LB * gsz + NW * NBW;
    auto row0_eval = [&](int bb) {
        const int i = bb * LB + (lane >> 1);
        if (lane < 2 * LB && i <= Lq.Q) eval_node(RZ + lane * NVP, wsing[i], true);
    };

    // first prefetch batch of the next latitude block: block 0's here, each
    // later one loaded at the end of the block before, so that its latency
    // hides behind that block's longitude sums
    double avn[PF];
    {
        const auto lf0 = gmem(Lq.lfrag + (long long)wv * SC::KW * 64 + lane);
#pragma unroll
        for (int u = 0; u < PF; ++u) avn[u] = (u < SC::KW) ? lf0[(long long)u * 64] : 0.0;
    }
    for (int b = 0; b < nblk; ++b) {
        if (SC::ROW0 && qg.l0 == 1 && b > 0 && wv == ((b - 1) & (NW - 1))) row0_eval(b - 1);
        // 3a. Legendre sums on MFMA: per degree column of this wave, a chain
        //     over n of (Pbar; dPbar at 8 latitudes) x (rotated coefficients).
        //     This wave's A fragments are contiguous in the table (zero past
        //     its last k-step), so they stream in batches independent of the
        //     column bookkeeping.
        {
            const auto lf = gmem(Lq.lfrag + ((long long)b * NW + wv) * SC::KW * 64 + lane);
            double av[2][PF];
#pragma unroll
            for (int u = 0; u < PF; ++u) av[0][u] = avn[u];
            int m = m_first, left = (m <= p) ? (p + 1 - m + 3) / 4 : 0;
            bool odd_step = (m_first / NW) & 1;
            dbl4 a = dbl4{0, 0, 0, 0};
            // 1 / sin theta at this lane's two latitudes (clamped past the last one)
            const double rs0 = rsin[min(b * LB + (lane >> 4), Lq.Q)];
            const double rs1 = rsin[min(b * LB + (lane >> 4) + 4, Lq.Q)];
#pragma unroll
            for (int g = 0; g < NBATCH; ++g) {
                if (g + 1 < NBATCH) {
#pragma unroll
                    for (int u = 0; u < PF; ++u) {
                        const int t = (g + 1) * PF + u;
                        av[(g + 1) & 1][u] = (t < SC::KW) ? lf[(long long)t * 64] : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const int t = g * PF + u;
                    if (t < SC::KW && left > 0) {
                        a = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g & 1][u], cB[t], a, 0, 0, 0);
                        if (--left == 0) {   // column finished: store it, go to the next one
                            store_col(m, a, rs0, rs1);
                            a = dbl4{0, 0, 0, 0};
                            m += odd_step ? dm1 : dm0;
                            odd_step = !odd_step;
                            left = (m <= p) ? (p + 1 - m + 3) / 4 : 0;
                        }
                    }
                }
            }
            if (b + 1 < nblk) {
                const auto lfn = lf + (long long)NW * SC::KW * 64;   // block b + 1, this wave
#pragma unroll
                for (int u = 0; u < PF; ++u) avn[u] = (u < SC::KW) ? lfn[(long long)u * 64] : 0.0;
            }
        }
        __syncthreads();

        // 3b/3c. per latitude of the block owned by this wave: longitude
        //     sums of its row tile on MFMA (four term-group chains), node
        //     values through the wave's own LDS buffer (64 nodes: {l, H - l,
        //     H + l, N - l} x 16 rows), then one node per lane: kernels with
        //     the modified weights.
        if (dft_wave) {
            const int boff = (lane >> 4) * 16 + (lane & 15);
            // Four row tiles (p = 48): the two waves of a tile share a SIMD,
            // and with four latitudes each the first finished its sums well
            // before the second; taking five of the eight balances the pair
            // (67.6 -> 66.3 ms on the 64-drop workload).  Otherwise latitudes
            // are dealt round-robin over the waves of a tile.
            const bool split = qg.nTp == 4;
            const int ll0 = split ? (wv < 4 ? 0 : 5) : wv / qg.nTp;
            const int ll1 = split ? (wv < 4 ? 5 : LB) : LB;
            const int dll = split ? 1 : SC::NW / qg.nTp;
            int nmine = 0;                               // this wave's latitudes in the block
            for (int ll = ll0; ll < ll1 && b * LB + ll <= Lq.Q; ll += dll) ++nmine;
            // node of this lane; the four images coincide pairwise at l = 0 and at 2 l = H
            const int c4 = lane >> 4, l = qg.l0 + 16 * my_tile + (lane & 15);
            const bool node_ok = 2 * l <= qg.H &&
                                 (c4 == 0 || (c4 == 1 && 2 * l < qg.H) || (c4 == 2 && l > 0) ||
                                  (c4 == 3 && l > 0 && 2 * l < qg.H));
            dbl4 ec, es, oc, os;
            // longitude sums of latitude ll of the block, this wave's row tile:
            // k-steps up to the class maximum without guards (past a group's
            // last k-step the A fragment is zero and the B address is clamped
            // to the group's last k-step)
            auto chain = [&](int ll) {
                const double* G = R + ll * gsz + boff;
                ec = dbl4{0, 0, 0, 0};
                es = ec;
                oc = ec;
                os = ec;
                const int kl0 = qg.nk[0] - 1, kl1 = qg.nk[1] - 1, kl2 = qg.nk[2] - 1, kl3 = qg.nk[3] - 1;
                const int g0 = qg.base[0] / 4, g1 = qg.base[1] / 4, g2 = qg.base[2] / 4, g3 = qg.base[3] / 4;
#pragma unroll
                for (int ks = 0; ks < SC::KEC; ++ks) {
                    ec = __builtin_amdgcn_mfma_f64_16x16x4f64(aEC[ks], G[(g0 + min(ks, kl0)) * 64], ec, 0, 0, 0);
                    if (ks < SC::KES)
                        es = __builtin_amdgcn_mfma_f64_16x16x4f64(aES[ks < SC::KES ? ks : 0],
                                                                  G[(g1 + max(min(ks, kl1), 0)) * 64], es, 0, 0, 0);
                    if (ks < SC::KOC) {
                        oc = __builtin_amdgcn_mfma_f64_16x16x4f64(aOC[ks < SC::KOC ? ks : 0], G[(g2 + min(ks, kl2)) * 64],
                                                                  oc, 0, 0, 0);
                        os = __builtin_amdgcn_mfma_f64_16x16x4f64(aOS[ks < SC::KOC ? ks : 0], G[(g3 + min(ks, kl3)) * 64],
                                                                  os, 0, 0, 0);
                    }
                }
            };
            // node buffer <- the four images of the latitude in ec, es, oc, os
            // (record 16 c + row for the nodes c = 0..3 of the row), then this
            // lane's node values -> nv (registers: the buffer is then free)
            auto publish = [&](double* nv) {
                {
                    // lanes of the unused columns v >= NV write to spare slots
                    // past the records instead of branching around the stores
                    const int v = lane & 15;
                    const bool real = v < NV;
                    double* const dst = real ? NB + v : NB + 64 * NVP + (v - NV);
                    const int step = real ? NVP : 0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = (lane >> 4) + 4 * r;
                        const double s0 = ec[r] + oc[r], s1 = ec[r] - oc[r];
                        const double t0 = es[r] + os[r], t1 = es[r] - os[r];
                        dst[row * step] = s0 + t0;             // l
                        dst[(16 + row) * step] = s1 - t1;      // H - l
                        dst[(32 + row) * step] = s1 + t1;      // H + l
                        dst[(48 + row) * step] = s0 - t0;      // N - l
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int v = 0; v < NV; ++v) nv[v] = NB[lane * NVP + v];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            };
            // Software pipeline over a wave's two latitudes (p = 24, 32): the
            // second latitude's sums are issued to the matrix unit right before
            // the vector unit evaluates the kernels at the first latitude's
            // nodes, in one basic block, so the two overlap.  (p = 48 has no
            // registers to spare for it, p = 16 one latitude per wave and block.)
            double na[NV], nb[NV];
            if (PMAX <= 32 && nmine == 2) {
                // the weights are loaded unconditionally (both latitudes exist),
                // so no branch splits the block
                const double wa = wsing[b * LB + ll0], wb = wsing[b * LB + ll0 + dll];
                chain(ll0);
                publish(na);
                __builtin_amdgcn_sched_barrier(0);
                chain(ll0 + dll);
                eval_node(na, node_ok ? wa : 0.0, false);
                __builtin_amdgcn_sched_barrier(0);
                publish(nb);
                eval_node(nb, node_ok ? wb : 0.0, false);
            } else {
                for (int ll = ll0; ll < ll1; ll += dll) {
                    const int i = b * LB + ll;
                    if (i > Lq.Q) break;
                    const double* G = R + ll * gsz + boff;
                    dbl4 ec1 = dbl4{0, 0, 0, 0}, es1 = ec1, oc1 = ec1, os1 = ec1;
                    const int kl0 = qg.nk[0] - 1, kl1 = qg.nk[1] - 1, kl2 = qg.nk[2] - 1, kl3 = qg.nk[3] - 1;
                    const int g0 = qg.base[0] / 4, g1 = qg.base[1] / 4, g2 = qg.base[2] / 4, g3 = qg.base[3] / 4;
#pragma unroll
                    for (int ks = 0; ks < SC::KEC; ++ks) {
                        ec1 = __builtin_amdgcn_mfma_f64_16x16x4f64(aEC[ks], G[(g0 + min(ks, kl0)) * 64], ec1, 0, 0, 0);
                        if (ks < SC::KES)
                            es1 = __builtin_amdgcn_mfma_f64_16x16x4f64(aES[ks < SC::KES ? ks : 0],
                                                                       G[(g1 + max(min(ks, kl1), 0)) * 64], es1, 0, 0,
                                                                       0);
                        if (ks < SC::KOC) {
                            oc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(aOC[ks < SC::KOC ? ks : 0],
                                                                       G[(g2 + min(ks, kl2)) * 64], oc1, 0, 0, 0);
                            os1 = __builtin_amdgcn_mfma_f64_16x16x4f64(aOS[ks < SC::KOC ? ks : 0],
                                                                       G[(g3 + min(ks, kl3)) * 64], os1, 0, 0, 0);
                        }
                    }
                    // node buffer: record 16 c + row for the nodes c = 0..3 of the row
                    {
                        const int v = lane & 15;
                        if (v < NV) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int row = (lane >> 4) + 4 * r;
                                const double s0 = ec1[r] + oc1[r], s1 = ec1[r] - oc1[r];
                                const double t0 = es1[r] + os1[r], t1 = es1[r] - os1[r];
                                NB[row * NVP + v] = s0 + t0;             // l
                                NB[(16 + row) * NVP + v] = s1 - t1;      // H - l
                                NB[(32 + row) * NVP + v] = s1 + t1;      // H + l
                                NB[(48 + row) * NVP + v] = s0 - t0;      // N - l
                            }
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if (node_ok) eval_node(NB + lane * NVP, wsing[i], true);
                    // the buffer is rewritten for the next latitude
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
        }
        // 3d. when row 0 is apart: row 0 of latitude wv of the block, phi = 0
        //     and pi take EC + OC and EC - OC, the sums of the cos rows of even
        //     and odd m; lane (column v, part) sums every fourth row, shuffles
        //     add the parts; the two records go to the row-0 area.
        if (SC::ROW0 && qg.l0 == 1 && b * LB + wv <= Lq.Q) {
            const double* G = R + wv * gsz + (lane & 15);
            const int part = lane >> 4;
            double ecs = 0.0, ocs = 0.0;
            for (int k = 0; k < qg.nk[0]; ++k) ecs += G[(qg.base[0] + 4 * k + part) * 16];
            for (int k = 0; k < qg.nk[2]; ++k) ocs += G[(qg.base[2] + 4 * k + part) * 16];
            ecs += __shfl_xor(ecs, 16);
            ecs += __shfl_xor(ecs, 32);
            ocs += __shfl_xor(ocs, 16);
            ocs += __shfl_xor(ocs, 32);
            const int v = lane & 15;
            if (part < 2 && v < NV) RZ[(2 * wv + part) * NVP + v] = part ? ecs - ocs : ecs + ocs;
        }
        __syncthreads();  // Fourier blocks consumed before the next block's Legendre sums
    }
    if (SC::ROW0 && qg.l0 == 1 && nblk > 0 && wv == ((nblk - 1) & (NW - 1))) row0_eval(nblk - 1);
    for (int c = 0; c < 9; ++c) {
        const double sv = wave_sum_dpp(acc[c]);
        if (lane == 0) red[wv][c] = sv;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double sv = 0.0;
        for (int w = 0; w < NW; ++w) sv += red[w][threadIdx.x];
        const unsigned bit = threadIdx.x < 3 ? EHD_STOKES_SL : threadIdx.x < 6 ? EHD_STOKES_DL
                             : threadIdx.x == 6 ? EHD_LAP_SL : threadIdx.x == 7 ? EHD_LAP_DL
                                                                                : EHD_LAP_DLADJ;
        const bool mine = (threadIdx.x < 3 && HF) || (threadIdx.x >= 3 && threadIdx.x < 6 && (HF || HU)) ||
                          (threadIdx.x >= 6 && HS);
        if ((kinds & bit) && mine) raw[threadIdx.x * T + tg] = sv * kInv4Pi;
    }
}

// ---------------------------------------------------------------------------
// Far field: each thread TPT targets (rows t, t + 256, ...), sources streamed
// through LDS in tiles of one drop each (drop-aligned padding; a tile's
// entry in tile_info gives its drop and how many of its slots, rounded up to
// four, hold sources, and only those are loaded and summed), tiles split
// over blockIdx.y.  partial[chunk][comp][T] (unscaled).  TPT and the number
// of chunks are the tile-shape parameters the autotuner picks.
// ---------------------------------------------------------------------------
// FP64 far field: as the FP32 kernel below (kinds a template parameter,
// sources read two at a time as double2 broadcasts from each LDS record
// row), with absolute coordinates and plain FP64 sums.  The pair terms use
// 2/r and its powers (rsqrt2_newton); each output's power of two, and the
// double layer's -6, multiply the tile sums, and the Stokes single layer
// keeps its f/r and r^-3 parts in separate tile sums (2 and 8 times the
// terms).
template <int TPT, unsigned KM>
__device__ __forceinline__ void far64_block(const double* __restrict__ tx,
                                                    const double* __restrict__ tnrm,
                                                    const int* __restrict__ tdrop, long long T,
                                                    const double* __restrict__ src, long long Spad,
                                                    const int2* __restrict__ tile_info, int ntiles,
                                                    int tiles_per_chunk, double* __restrict__ partial, int bx, int by)
{
    constexpr bool wS = KM & EHD_STOKES_SL, wD = KM & EHD_STOKES_DL;
    constexpr bool wSL = KM & EHD_LAP_SL, wL = KM & EHD_LAP_DL, wK = KM & EHD_LAP_DLADJ;
    constexpr bool needN = wD || wL, needSig = wSL || wL || wK;
    __shared__ double2 sm[kRec64][kTile / 2];
    double* const smd = reinterpret_cast<double*>(&sm[0][0]);
    double x0[TPT], y0[TPT], z0[TPT], n0x[TPT], n0y[TPT], n0z[TPT], acc[TPT][9];
    int myd[TPT];
    long long tt[TPT];
    for (int q = 0; q < TPT; ++q) {
        tt[q] = (long long)bx * blockDim.x * TPT + q * blockDim.x + threadIdx.x;
        const bool valid = tt[q] < T;
        const long long u = valid ? tt[q] : 0;
        x0[q] = tx[u]; y0[q] = tx[T + u]; z0[q] = tx[2 * T + u];
        n0x[q] = tnrm[u]; n0y[q] = tnrm[T + u]; n0z[q] = tnrm[2 * T + u];
        myd[q] = valid ? tdrop[u] : -1;
        for (int c = 0; c < 9; ++c) acc[q][c] = 0.0;
    }
    // targets are stored drop by drop: a block whose first and last targets
    // lie on one drop skips that drop's tiles whole
    const long long tb0 = (long long)bx * blockDim.x * TPT, tb1 = min(T - 1, tb0 + (long long)blockDim.x * TPT - 1);
    const int bdrop = tdrop[tb0] == tdrop[tb1] ? tdrop[tb0] : -1;
    const int t0 = by * tiles_per_chunk, t1 = min(ntiles, t0 + tiles_per_chunk);
    for (int tile = t0; tile < t1; ++tile) {
        const int2 ti = tile_info[tile];          // (drop, sources in the tile)
        if (ti.x == bdrop) continue;              // uniform over the block
        const long long s = (long long)tile * kTile + threadIdx.x;
        if ((int)threadIdx.x < ti.y)
            for (int r = 0; r < kRec64; ++r) smd[r * kTile + threadIdx.x] = src[r * Spad + s];
        __syncthreads();
        const int sd = ti.x;
        bool other = false;   // some target of this thread is not on the tile's drop
        for (int k = 0; k < TPT; ++k) other = other || (sd != myd[k]);
        double a[TPT][9], b[TPT][3];
        for (int k = 0; k < TPT; ++k) {
            for (int c = 0; c < 9; ++c) a[k][c] = 0.0;
            for (int c = 0; c < 3; ++c) b[k][c] = 0.0;
        }
        for (int q2 = 0; q2 < (other ? ti.y / 2 : 0); ++q2) {
            const double2 X = sm[0][q2], Y = sm[1][q2], Z = sm[2][q2];
            double2 NX, NY, NZ, F0, F1, F2, U0, U1, U2, SG;
            if constexpr (needN) { NX = sm[3][q2]; NY = sm[4][q2]; NZ = sm[5][q2]; }
            if constexpr (wS) { F0 = sm[7][q2]; F1 = sm[8][q2]; F2 = sm[9][q2]; }
            if constexpr (wD) { U0 = sm[10][q2]; U1 = sm[11][q2]; U2 = sm[12][q2]; }
            if constexpr (needSig) SG = sm[13][q2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const double xs = j ? X.y : X.x, ys = j ? Y.y : Y.x, zs = j ? Z.y : Z.x;
#pragma unroll
                for (int k = 0; k < TPT; ++k) {
                    const double hx = x0[k] - xs, hy = y0[k] - ys, hz = z0[k] - zs;
                    const double r2 = fma(hx, hx, fma(hy, hy, hz * hz));
                    // 2/r, 4/r^2, 8/r^3
                    const double ir = rsqrt2_newton(r2), ir2 = ir * ir, ir3 = ir * ir2;
                    // both double layers carry (h.n) / r^3
                    double hn3 = 0.0;
                    if constexpr (needN)
                        hn3 = fma(hx, j ? NX.y : NX.x, fma(hy, j ? NY.y : NY.x, hz * (j ? NZ.y : NZ.x))) * ir3;
                    if constexpr (wS) {
                        const double f0 = j ? F0.y : F0.x, f1 = j ? F1.y : F1.x, f2 = j ? F2.y : F2.x;
                        const double hf = fma(hx, f0, fma(hy, f1, hz * f2)) * ir3;
                        a[k][0] = fma(f0, ir, a[k][0]);
                        a[k][1] = fma(f1, ir, a[k][1]);
                        a[k][2] = fma(f2, ir, a[k][2]);
                        b[k][0] = fma(hx, hf, b[k][0]);
                        b[k][1] = fma(hy, hf, b[k][1]);
                        b[k][2] = fma(hz, hf, b[k][2]);
                    }
                    if constexpr (wD) {
                        const double hu =
                            fma(hx, j ? U0.y : U0.x, fma(hy, j ? U1.y : U1.x, hz * (j ? U2.y : U2.x)));
                        const double tq = (hu * ir2) * hn3;
                        a[k][3] = fma(tq, hx, a[k][3]);
                        a[k][4] = fma(tq, hy, a[k][4]);
                        a[k][5] = fma(tq, hz, a[k][5]);
                    }
                    if constexpr (needSig) {
                        const double sg = j ? SG.y : SG.x;
                        if constexpr (wSL) a[k][6] = fma(sg, ir, a[k][6]);
                        if constexpr (wL) a[k][7] = fma(sg, hn3, a[k][7]);
                        if constexpr (wK)
                            a[k][8] = fma(sg * fma(hx, n0x[k], fma(hy, n0y[k], hz * n0z[k])), ir3, a[k][8]);
                    }
                }
            }
        }
        for (int k = 0; k < TPT; ++k) {
            if (sd == myd[k]) continue;      // own drop: tile not counted
            // powers of two of 2/r: S 2 and 8, D 32 (with its -6), S_L 2, L and K* 8
            for (int c = 0; c < 3; ++c) acc[k][c] += fma(0.125, b[k][c], 0.5 * a[k][c]);
            for (int c = 3; c < 6; ++c) acc[k][c] += -0.1875 * a[k][c];
            acc[k][6] += 0.5 * a[k][6];
            acc[k][7] += 0.125 * a[k][7];
            acc[k][8] += 0.125 * a[k][8];
        }
        __syncthreads();
    }
    for (int k = 0; k < TPT; ++k)
        if (tt[k] < T)
            for (int c = 0; c < 9; ++c) partial[((long long)by * 9 + c) * T + tt[k]] = acc[k][c];
}

// Work items (target block bx, chunk by) = (vb % nbx, vb / nbx) for vb in
// [vb0, vb1), dealt to the blocks of the grid in turn: an ordinary launch has
// one block per item, a persistent one fewer blocks that loop.
template <int TPT, unsigned KM>
__global__ __launch_bounds__(kThreads) void k_far64(const double* __restrict__ tx, const double* __restrict__ tnrm,
                                                    const int* __restrict__ tdrop, long long T,
                                                    const double* __restrict__ src, long long Spad,
                                                    const int2* __restrict__ tile_info, int ntiles,
                                                    int tiles_per_chunk, double* __restrict__ partial, int nbx,
                                                    int vb0, int vb1)
{
    for (int vb = vb0 + (int)blockIdx.x; vb < vb1; vb += (int)gridDim.x)
        far64_block<TPT, KM>(tx, tnrm, tdrop, T, src, Spad, tile_info, ntiles, tiles_per_chunk, partial, vb % nbx,
                             vb / nbx);
}

// FP32 far field: the kinds KM are a template parameter (no per-interaction
// branches), sources are read four at a time as float4 from each LDS record
// row (one broadcast read per record and four sources).  Targets are taken
// relative to the centre of the tile's drop in FP64 and split into FP32
// high and low parts (h = (a - x_s) + b), the per-tile sums are FP32 and
// the tile sums are added with Kahan compensation.  The double-layer
// factor -6 is applied to the tile sums.
template <int TPT, unsigned KM>
__device__ __forceinline__ void far32_block(const double* __restrict__ tx,
                                                    const double* __restrict__ tnrm,
                                                    const int* __restrict__ tdrop, long long T,
                                                    const float* __restrict__ src, long long Spad,
                                                    const int2* __restrict__ tile_info,
                                                    const double* __restrict__ dcentre, int ntiles,
                                                    int tiles_per_chunk, double* __restrict__ partial, int bx, int by)
{
    constexpr bool wS = KM & EHD_STOKES_SL, wD = KM & EHD_STOKES_DL;
    constexpr bool wSL = KM & EHD_LAP_SL, wL = KM & EHD_LAP_DL, wK = KM & EHD_LAP_DLADJ;
    constexpr bool needN = wD || wL, needSig = wSL || wL || wK;
    __shared__ float4 sm[kRec32][kTile / 4];
    float* const smf = reinterpret_cast<float*>(&sm[0][0]);
    double X0[TPT], Y0[TPT], Z0[TPT];
    float n0x[TPT], n0y[TPT], n0z[TPT], sum[TPT][9], cmp[TPT][9];
    int myd[TPT];
    long long tt[TPT];
    for (int q = 0; q < TPT; ++q) {
        tt[q] = (long long)bx * blockDim.x * TPT + q * blockDim.x + threadIdx.x;
        const bool valid = tt[q] < T;
        const long long u = valid ? tt[q] : 0;
        X0[q] = tx[u]; Y0[q] = tx[T + u]; Z0[q] = tx[2 * T + u];
        n0x[q] = (float)tnrm[u]; n0y[q] = (float)tnrm[T + u]; n0z[q] = (float)tnrm[2 * T + u];
        myd[q] = valid ? tdrop[u] : -1;
        for (int c = 0; c < 9; ++c) { sum[q][c] = 0.0f; cmp[q][c] = 0.0f; }
    }
    // targets are stored drop by drop: a block whose first and last targets
    // lie on one drop skips that drop's tiles whole
    const long long tb0 = (long long)bx * blockDim.x * TPT, tb1 = min(T - 1, tb0 + (long long)blockDim.x * TPT - 1);
    const int bdrop = tdrop[tb0] == tdrop[tb1] ? tdrop[tb0] : -1;
    const int t0 = by * tiles_per_chunk, t1 = min(ntiles, t0 + tiles_per_chunk);
    for (int tile = t0; tile < t1; ++tile) {
        const int2 ti = tile_info[tile];          // (drop, sources in the tile)
        if (ti.x == bdrop) continue;              // uniform over the block
        const long long s = (long long)tile * kTile + threadIdx.x;
        if ((int)threadIdx.x < ti.y)
            for (int r = 0; r < kRec32; ++r) smf[r * kTile + threadIdx.x] = src[r * Spad + s];
        __syncthreads();
        const int sd = ti.x;
        bool other = false;   // some target of this thread is not on the tile's drop
        for (int k = 0; k < TPT; ++k) other = other || (sd != myd[k]);
        float ax[TPT], ay[TPT], az[TPT], bx[TPT], by[TPT], bz[TPT], a[TPT][9];
        const double* cj = dcentre + 4 * sd;            // centre, (2 radius)^2 of the tile's drop
        bool far_all = true;
        for (int k = 0; k < TPT; ++k) {
            const double dx = X0[k] - cj[0], dy = Y0[k] - cj[1], dz = Z0[k] - cj[2];
            ax[k] = (float)dx; ay[k] = (float)dy; az[k] = (float)dz;
            bx[k] = (float)(dx - ax[k]); by[k] = (float)(dy - ay[k]); bz[k] = (float)(dz - az[k]);
            far_all = far_all && (tt[k] >= T || dx * dx + dy * dy + dz * dz >= cj[3]);
            for (int c = 0; c < 9; ++c) a[k][c] = 0.0f;
        }
        // Targets at least two drop radii from the drop's centre have
        // |d| <= 2 |x0 - x| for every source x: the FP32 head of d alone
        // then keeps each term's relative error within a few roundings, and
        // the wave skips the tail (3 of 36 instructions per pair).
        const bool tail = !__all(far_all);
        auto pairs = [&](auto with_tail) {
        constexpr bool TAIL = decltype(with_tail)::value;
        for (int q4 = 0; q4 < (other ? ti.y / 4 : 0); ++q4) {
            const float4 X = sm[0][q4], Y = sm[1][q4], Z = sm[2][q4];
            float4 NX, NY, NZ, F0, F1, F2, U0, U1, U2, SG;
            if constexpr (needN) { NX = sm[3][q4]; NY = sm[4][q4]; NZ = sm[5][q4]; }
            if constexpr (wS) { F0 = sm[6][q4]; F1 = sm[7][q4]; F2 = sm[8][q4]; }
            if constexpr (wD) { U0 = sm[9][q4]; U1 = sm[10][q4]; U2 = sm[11][q4]; }
            if constexpr (needSig) SG = sm[12][q4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
#pragma unroll
                for (int k = 0; k < TPT; ++k) {
                    float hx = ax[k] - X[j], hy = ay[k] - Y[j], hz = az[k] - Z[j];
                    if constexpr (TAIL) { hx += bx[k]; hy += by[k]; hz += bz[k]; }
                    const float r2 = fmaf(hx, hx, fmaf(hy, hy, hz * hz));
                    const float ir = __frsqrt_rn(r2), ir2 = ir * ir, ir3 = ir * ir2;
                    float hn3 = 0.0f;   // (h.n) / r^3, shared by both double layers
                    if constexpr (needN) hn3 = fmaf(hx, NX[j], fmaf(hy, NY[j], hz * NZ[j])) * ir3;
                    if constexpr (wS) {
                        const float hf = fmaf(hx, F0[j], fmaf(hy, F1[j], hz * F2[j])) * ir3;
                        a[k][0] = fmaf(hx, hf, fmaf(F0[j], ir, a[k][0]));
                        a[k][1] = fmaf(hy, hf, fmaf(F1[j], ir, a[k][1]));
                        a[k][2] = fmaf(hz, hf, fmaf(F2[j], ir, a[k][2]));
                    }
                    if constexpr (wD) {
                        const float hu = fmaf(hx, U0[j], fmaf(hy, U1[j], hz * U2[j]));
                        const float tq = (hu * ir2) * hn3;
                        a[k][3] = fmaf(tq, hx, a[k][3]);
                        a[k][4] = fmaf(tq, hy, a[k][4]);
                        a[k][5] = fmaf(tq, hz, a[k][5]);
                    }
                    if constexpr (wSL) a[k][6] = fmaf(SG[j], ir, a[k][6]);
                    if constexpr (wL) a[k][7] = fmaf(SG[j], hn3, a[k][7]);
                    if constexpr (wK)
                        a[k][8] = fmaf(SG[j] * fmaf(hx, n0x[k], fmaf(hy, n0y[k], hz * n0z[k])), ir3, a[k][8]);
                }
            }
        }
        };
        if (tail) pairs(std::true_type{});
        else pairs(std::false_type{});
        for (int k = 0; k < TPT; ++k) {
            if (sd == myd[k]) continue;      // own drop: tile not counted
            for (int c = 3; c < 6; ++c) a[k][c] *= -6.0f;
            for (int c = 0; c < 9; ++c) {    // Kahan
                const float y = a[k][c] - cmp[k][c];
                const float tsum = sum[k][c] + y;
                cmp[k][c] = (tsum - sum[k][c]) - y;
                sum[k][c] = tsum;
            }
        }
        __syncthreads();
    }
    for (int k = 0; k < TPT; ++k)
        if (tt[k] < T)
            for (int c = 0; c < 9; ++c)
                partial[((long long)by * 9 + c) * T + tt[k]] = (double)sum[k][c] - (double)cmp[k][c];
}

// Work items as for k_far64.
template <int TPT, unsigned KM>
__global__ __launch_bounds__(kThreads) void k_far32(const double* __restrict__ tx, const double* __restrict__ tnrm,
                                                    const int* __restrict__ tdrop, long long T,
                                                    const float* __restrict__ src, long long Spad,
                                                    const int2* __restrict__ tile_info,
                                                    const double* __restrict__ dcentre, int ntiles,
                                                    int tiles_per_chunk, double* __restrict__ partial, int nbx,
                                                    int vb0, int vb1)
{
    for (int vb = vb0 + (int)blockIdx.x; vb < vb1; vb += (int)gridDim.x)
        far32_block<TPT, KM>(tx, tnrm, tdrop, T, src, Spad, tile_info, dcentre, ntiles, tiles_per_chunk, partial,
                             vb % nbx, vb / nbx);
}

// Outputs: rows of the requested kinds, scaled far sums added to (or written
// beside) the self part.
struct RowMap {
    int n;
    int comp[9];
};

__global__ void k_combine(const double* __restrict__ raw_self, const double* __restrict__ partial,
                          int nchunk, long long T, RowMap rows, double* __restrict__ self_out,
                          double* __restrict__ far_out)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    for (int r = 0; r < rows.n; ++r) {
        const int c = rows.comp[r];
        double f = 0.0;
        for (int ch = 0; ch < nchunk; ++ch) f += partial[((long long)ch * 9 + c) * T + t];
        f *= kInv4Pi;
        const double s = raw_self[(long long)c * T + t];
        if (far_out) {
            self_out[(long long)r * T + t] = s;
            far_out[(long long)r * T + t] = f;
        } else {
            self_out[(long long)r * T + t] = s + f;
        }
    }
}

// Galerkin analysis: one block per (drop, n(n+1)/2+m) coefficient group,
// (y, Y_nm) = sum_j sum_k (2pi/nlon) w_j y_jk Pbar_n^m(t_j) e^{-i m phi_k}.
__global__ void k_analyze(const DropInfo* __restrict__ drops, const LegTab* __restrict__ legs,
                          const int2* __restrict__ items, int nf, const double* __restrict__ grid,
                          long long T, double* __restrict__ coef)
{
    const int2 it = items[blockIdx.x];
    const DropInfo D = drops[it.x];
    const LegTab L = legs[D.leg_pp];
    const int p = L.p, kk = it.y;
    const int n = tri_n(kk), m = kk - n * (n + 1) / 2;
    const long nc = ncoef(p);
    const int npts = (L.Q + 1) * L.nlon;
    __shared__ double rr[kThreads / 64][2];
    for (int f = 0; f < nf; ++f) {
        double ar = 0.0, ai = 0.0;
        for (int q = threadIdx.x; q < npts; q += blockDim.x) {
            const int j = q / L.nlon, l = q % L.nlon;
            const double y = grid[(long long)f * T + D.toff + q] * L.wq[j] * L.P[(long long)j * nc + kk];
            const double* tr = L.trig + ((long long)l * (p + 1) + m) * 2;
            ar += y * tr[0];
            ai -= y * tr[1];
        }
        ar = wave_sum(ar);
        ai = wave_sum(ai);
        if ((threadIdx.x & 63) == 0) { rr[threadIdx.x >> 6][0] = ar; rr[threadIdx.x >> 6][1] = ai; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double sr = 0.0, si = 0.0;
            for (int w = 0; w < (int)(blockDim.x / 64); ++w) { sr += rr[w][0]; si += rr[w][1]; }
            double* cb = coef + (long long)nf * D.coff + (long long)f * 2 * nc;
            cb[2 * kk] = sr;
            cb[2 * kk + 1] = (m == 0) ? 0.0 : si;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Nearly singular targets (Sec. 2.1, the interpolation approach): for a
// target x0 closer than delta to the surface of another drop j, drop j's
// contribution is replaced by the value at x0 of the polynomial through
//   s = 0:   the limit from outside at the closest surface point y, i.e. the
//            on-surface singular-rule values of drop j projected to degree p
//            and evaluated at y, plus the jumps (S, S_L continuous; D: -u(y);
//            L: +sigma(y)/2; K* with the target normal n0:
//            -n0 . grad_S S_L(y) + (K*(y) + sigma(y)/2)(n0 . n_y));
//   s = s_k: drop j's regular-rule sums at y + s_k nu on a finer check grid,
//            s_k = s_check (1 + k/2), k = 0..m-1, nu = (x0 - y)/|x0 - y|;
// at s = |x0 - y|; the regular-rule value of drop j at x0 (what the far sum
// added) is subtracted.
// ---------------------------------------------------------------------------
struct NearPair {
    int t, j;                 // target, source drop
    double th, ph;            // closest point parameters on drop j
    double y[3], ny[3], xt[3], xp[3], nu[3];   // point, unit normal, d/dtheta, d/dphi, line direction
    double st;                // |x0 - y|
    long long legoff;         // Pbar then dPbar/dtheta at cos(th): 2 ncoef(p_j) doubles
};

// Check-grid geometry from synthesized x, x_theta, x_phi/sin: records
// x(3) n(3) w(1) in the layout of the far-source records.
__global__ void k_fine_geom(const DropInfo* __restrict__ fdrops, const LegTab* __restrict__ flegs,
                            const int* __restrict__ node_drop, const double* __restrict__ syn, long long N,
                            double* __restrict__ rec)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const DropInfo D = fdrops[node_drop[s]];
    const LegTab L = flegs[D.leg_pf];
    const int i = (int)((s - D.soff) / L.nlon);
    double xt[3], xp[3];
    for (int c = 0; c < 3; ++c) {
        rec[c * N + s] = syn[c * N + s];
        xt[c] = syn[(3 + c) * N + s];
        xp[c] = syn[(6 + c) * N + s];
    }
    const double cx = xt[1] * xp[2] - xt[2] * xp[1];
    const double cy = xt[2] * xp[0] - xt[0] * xp[2];
    const double cz = xt[0] * xp[1] - xt[1] * xp[0];
    const double J = sqrt(cx * cx + cy * cy + cz * cz);
    rec[3 * N + s] = cx / J;
    rec[4 * N + s] = cy / J;
    rec[5 * N + s] = cz / J;
    rec[6 * N + s] = L.wq[i] * J;
}

// Weighted densities of the check-grid records (u = f when no u is given).
__global__ void k_fine_dens(const double* __restrict__ synf, const double* __restrict__ synu,
                            const double* __restrict__ syns, long long N, double* __restrict__ rec)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const double w = rec[6 * N + s];
    for (int c = 0; c < 3; ++c) {
        const double f = synf ? w * synf[c * N + s] : 0.0;
        rec[(7 + c) * N + s] = f;
        rec[(10 + c) * N + s] = synu ? w * synu[c * N + s] : f;
    }
    rec[13 * N + s] = syns ? w * syns[s] : 0.0;
}

// Exterior limits at the closest points, one block per pair.  selfc: the
// projected on-surface self values (9 fields per drop); u: u or f (3 fields),
// sig (1 field), each in the packed per-drop layout; lim[pair][9].
__global__ __launch_bounds__(kThreads) void k_near_limit(const NearPair* __restrict__ pairs,
                                                         const DropInfo* __restrict__ drops,
                                                         const double* __restrict__ legv,
                                                         const double* __restrict__ selfc,
                                                         const double* __restrict__ ucoef,
                                                         const double* __restrict__ scoef,
                                                         const double* __restrict__ tnrm, long long T,
                                                         double* __restrict__ lim)
{
    constexpr int NA = 9 + 3 + 1 + 2;     // self fields, u, sigma, d/dtheta and d/dphi of S_L
    const NearPair P = pairs[blockIdx.x];
    const DropInfo D = drops[P.j];
    const int p = D.p;
    const long nc = ncoef(p);
    const double* Pb = legv + P.legoff;
    const double* dPb = Pb + nc;
    double acc[NA];
    for (int a = 0; a < NA; ++a) acc[a] = 0.0;
    for (long k = threadIdx.x; k < nc; k += blockDim.x) {
        const int n = tri_n((int)k), m = (int)k - n * (n + 1) / 2;
        double sm, cm;
        sincos(m * P.ph, &sm, &cm);
        const double mult = m ? 2.0 : 1.0, pv = Pb[k], dv = dPb[k];
        auto re = [&](const double* c) { return c[2 * k] * cm - (m ? c[2 * k + 1] : 0.0) * sm; };
        for (int f = 0; f < 9; ++f) acc[f] += mult * pv * re(selfc + 9 * D.coff + f * 2 * nc);
        for (int c = 0; c < 3; ++c) acc[9 + c] += mult * pv * re(ucoef + 3 * D.coff + c * 2 * nc);
        acc[12] += mult * pv * re(scoef + D.coff);
        const double* sl = selfc + 9 * D.coff + 6 * 2 * nc;
        acc[13] += mult * dv * re(sl);
        acc[14] -= mult * m * pv * (sl[2 * k] * sm + (m ? sl[2 * k + 1] : 0.0) * cm);
    }
    __shared__ double red[kThreads / 64][NA];
    for (int a = 0; a < NA; ++a) {
        const double v = wave_sum(acc[a]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][a] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double v[NA];
    for (int a = 0; a < NA; ++a) {
        v[a] = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) v[a] += red[w][a];
    }
    const double E = P.xt[0] * P.xt[0] + P.xt[1] * P.xt[1] + P.xt[2] * P.xt[2];
    const double F = P.xt[0] * P.xp[0] + P.xt[1] * P.xp[1] + P.xt[2] * P.xp[2];
    const double G = P.xp[0] * P.xp[0] + P.xp[1] * P.xp[1] + P.xp[2] * P.xp[2];
    const double iW2 = 1.0 / (E * G - F * F);
    const double a = (G * v[13] - F * v[14]) * iW2, b = (E * v[14] - F * v[13]) * iW2;
    double n0g = 0.0, n0n = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double n0 = tnrm[c * T + P.t];
        n0g += n0 * (a * P.xt[c] + b * P.xp[c]);
        n0n += n0 * P.ny[c];
    }
    double* o = lim + 9 * (long long)blockIdx.x;
    for (int c = 0; c < 3; ++c) {
        o[c] = v[c];
        o[3 + c] = v[3 + c] - v[9 + c];
    }
    o[6] = v[6];
    o[7] = v[7] + 0.5 * v[12];
    o[8] = -n0g + (v[8] + 0.5 * v[12]) * n0n;
}

// Kernels of drop j's regular rule at a point p (normal n0 for K*), added to
// a[9] for one source record (x, n, w f, w u, w sigma).
__device__ __forceinline__ void near_pair_sum(const double* p, const double* n0, double sx, double sy, double sz,
                                              double nx, double ny, double nz, double f0, double f1, double f2,
                                              double u0, double u1, double u2, double sg, double* a)
{
    const double hx = p[0] - sx, hy = p[1] - sy, hz = p[2] - sz;
    const double ir = rsqrt_nr(hx * hx + hy * hy + hz * hz), ir2 = ir * ir, ir3 = ir * ir2;
    const double hn = hx * nx + hy * ny + hz * nz;
    const double hf = (hx * f0 + hy * f1 + hz * f2) * ir3;
    a[0] += f0 * ir + hx * hf;
    a[1] += f1 * ir + hy * hf;
    a[2] += f2 * ir + hz * hf;
    const double tq = -6.0 * (hx * u0 + hy * u1 + hz * u2) * hn * ir3 * ir2;
    a[3] += tq * hx;
    a[4] += tq * hy;
    a[5] += tq * hz;
    a[6] += sg * ir;
    a[7] += sg * hn * ir3;
    a[8] += sg * (hx * n0[0] + hy * n0[1] + hz * n0[2]) * ir3;
}

// Check-point sums: block (pair, chunk) walks chunk `chunk` of kNearSplit
// ranges of drop j's check grid; each thread takes every kThreads-th record
// straight from memory (coalesced) and adds its kernels at four check points
// y + s_k nu at a time, so that one read of a record serves four points.
// out[pair][chunk][k][9] (1/(4 pi) applied); the chunks are added in order
// by k_near_apply.
__global__ __launch_bounds__(kThreads) void k_near_check(const NearPair* __restrict__ pairs, int m, double sc,
                                                         const double* __restrict__ frec, long long Nf,
                                                         const long long* __restrict__ foff,
                                                         const int* __restrict__ fidx,
                                                         const double* __restrict__ tnrm, long long T,
                                                         double* __restrict__ out)
{
    constexpr int G = 4;                                  // check points per pass over the records
    __shared__ double red[kThreads / 64][G * 9];
    const int pi = blockIdx.x, lane = threadIdx.x & 63;
    const NearPair P = pairs[pi];
    double n0[3];
    for (int c = 0; c < 3; ++c) n0[c] = tnrm[c * T + P.t];
    const int fd = fidx[P.j];
    const long long len = foff[fd + 1] - foff[fd];
    const long long c0 = foff[fd] + len * blockIdx.y / kNearSplit, c1 = foff[fd] + len * (blockIdx.y + 1) / kNearSplit;
    for (int k0 = 0; k0 < m; k0 += G) {
        double pt[G][3], a[G][9];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            for (int c = 0; c < 3; ++c) pt[g][c] = P.y[c] + sc * (1.0 + 0.5 * (k0 + g)) * P.nu[c];
            for (int c = 0; c < 9; ++c) a[g][c] = 0.0;
        }
        // record rows: x 0-2, n 3-5, (w 6), w f 7-9, w u 10-12, w sigma 13
        for (long long s = c0 + threadIdx.x; s < c1; s += kThreads) {
            const double sx = frec[s], sy = frec[Nf + s], sz = frec[2 * Nf + s];
            const double nx = frec[3 * Nf + s], ny = frec[4 * Nf + s], nz = frec[5 * Nf + s];
            const double f0 = frec[7 * Nf + s], f1 = frec[8 * Nf + s], f2 = frec[9 * Nf + s];
            const double u0 = frec[10 * Nf + s], u1 = frec[11 * Nf + s], u2 = frec[12 * Nf + s];
            const double sg = frec[13 * Nf + s];
#pragma unroll
            for (int g = 0; g < G; ++g)
                near_pair_sum(pt[g], n0, sx, sy, sz, nx, ny, nz, f0, f1, f2, u0, u1, u2, sg, a[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
            for (int c = 0; c < 9; ++c) {
                const double v = wave_sum(a[g][c]);
                if (lane == 0) red[threadIdx.x >> 6][g * 9 + c] = v;
            }
        __syncthreads();
        if (threadIdx.x < G * 9 && k0 + threadIdx.x / 9 < m) {
            double v = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) v += red[w][threadIdx.x];
            const int k = k0 + threadIdx.x / 9, c = threadIdx.x % 9;
            out[(((long long)pi * kNearSplit + blockIdx.y) * (m + 1) + k) * 9 + c] = v * kInv4Pi;
        }
        __syncthreads();   // red is rewritten by the next pass
    }
}

// Drop j's regular-rule value at the target x0 on its far-grid records (what
// the far sum added), one block per pair, into the chunk-0 slot of k = m.
__global__ __launch_bounds__(kThreads) void k_near_plain(const NearPair* __restrict__ pairs, int m,
                                                         const double* __restrict__ src, long long Spad,
                                                         const DropInfo* __restrict__ drops,
                                                         const double* __restrict__ tx,
                                                         const double* __restrict__ tnrm, long long T,
                                                         double* __restrict__ out)
{
    const int pi = blockIdx.x;
    const NearPair P = pairs[pi];
    const DropInfo D = drops[P.j];
    double pt[3], n0[3];
    for (int c = 0; c < 3; ++c) {
        pt[c] = tx[c * T + P.t];
        n0[c] = tnrm[c * T + P.t];
    }
    double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (long long s = D.soff + threadIdx.x; s < D.soff + D.ns; s += blockDim.x)
        near_pair_sum(pt, n0, src[s], src[Spad + s], src[2 * Spad + s], src[3 * Spad + s], src[4 * Spad + s],
                      src[5 * Spad + s], src[7 * Spad + s], src[8 * Spad + s], src[9 * Spad + s], src[10 * Spad + s],
                      src[11 * Spad + s], src[12 * Spad + s], src[13 * Spad + s], a);
    __shared__ double red[kThreads / 64][9];
    for (int c = 0; c < 9; ++c) {
        const double v = wave_sum(a[c]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double v = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) v += red[w][threadIdx.x];
        out[((long long)pi * kNearSplit * (m + 1) + m) * 9 + threadIdx.x] = v * kInv4Pi;
    }
}

// Lagrange interpolation and the correction of the output rows, one block
// per pair: thread (k, c) adds the chunks of check point k (k = m: the plain
// value at the target) in order, then thread r combines row r's values in
// order of k (pairs sharing a target add atomically).
__global__ __launch_bounds__(128) void k_near_apply(const NearPair* __restrict__ pairs, int m, double sc,
                                                    const double* __restrict__ lim, const double* __restrict__ chk,
                                                    RowMap rows, double* __restrict__ corr)
{
    __shared__ double sk[(kNearMaxM + 1) * 9];
    const int pi = blockIdx.x;
    const double* c0 = chk + (long long)pi * kNearSplit * (m + 1) * 9;
    for (int i = threadIdx.x; i < (m + 1) * 9; i += blockDim.x) {
        const int k = i / 9, c = i % 9;
        double v = 0.0;
        for (int h = 0; h < kNearSplit; ++h) v += c0[(h * (m + 1) + k) * 9 + c];
        sk[i] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x >= rows.n) return;
    const NearPair P = pairs[pi];
    double nodes[kNearMaxM + 1];
    nodes[0] = 0.0;
    for (int k = 0; k < m; ++k) nodes[k + 1] = sc * (1.0 + 0.5 * k);
    double w[kNearMaxM + 1];
    for (int k = 0; k <= m; ++k) {
        double l = 1.0;
        for (int i = 0; i <= m; ++i)
            if (i != k) l *= (P.st - nodes[i]) / (nodes[k] - nodes[i]);
        w[k] = l;
    }
    const int r = threadIdx.x, c = rows.comp[r];
    double v = w[0] * lim[9 * (long long)pi + c];
    for (int k = 0; k <= m; ++k) v += k < m ? w[k + 1] * sk[k * 9 + c] : -sk[k * 9 + c];
    corr[9 * (long long)pi + r] = v;
}

// Adds each corrected target's pair corrections to its output rows: one
// thread per (target, row), the target's pairs (consecutive: pairs are kept
// in target order) summed in their stored order, so the result does not
// depend on scheduling.
__global__ void k_near_gather(const int* __restrict__ tstart, const int* __restrict__ tlist, int ntgt,
                              const double* __restrict__ corr, RowMap rows, long long T, double* __restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)ntgt * rows.n) return;
    const int u = (int)(i / rows.n), r = (int)(i % rows.n);
    double v = 0.0;
    for (int pi = tstart[u]; pi < tstart[u + 1]; ++pi) v += corr[9 * (long long)pi + r];
    out[(long long)r * T + tlist[u]] += v;
}

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================
struct ehd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int max_lds = 65536;
    int ncu = 256;                       // compute units (looping far-field blocks in overlap mode)

    // drops
    int nd = 0, grid_mode = 0;
    std::vector<int> p, qs, qf;
    std::vector<DropInfo> info;
    long long T = 0, Spad = 0, ncoef_total = 0;  // ncoef_total: doubles per field
    int ntiles = 0;
    // singular self-interaction work, by degree class (PMAX 16, 24, 32, 48):
    // targets of the class's drops, most expensive drops first
    std::vector<int> self_order_h;
    int cls_off[5] = {0, 0, 0, 0, 0};
    std::vector<int> cls_drops[4];

    // device buffers
    std::vector<void*> allocs;
    DropInfo* d_info = nullptr;
    LegTab* d_legs = nullptr;
    WigTab* d_wigs = nullptr;
    double* d_x = nullptr;           // own copy of x coefficients
    double* d_tx = nullptr;          // [3][T]
    double* d_tn = nullptr;          // [3][T]
    int* d_tdrop = nullptr;          // [T]
    int* d_order = nullptr;          // [T] self work order
    int* d_slot_drop = nullptr;      // [Spad]
    int2* d_tile_info = nullptr;     // [ntiles] (drop, sources in the tile rounded up to 4)
    double* d_centre = nullptr;      // [4*nd]: centre, (2 radius)^2
    double* d_src64 = nullptr;       // [kRec64][Spad]
    float* d_src32 = nullptr;        // [kRec32][Spad]
    double* d_syn = nullptr;         // synthesis scratch [9][max(T,Spad)]
    long long syn_stride = 0;
    double* d_raw = nullptr;         // [9][T]
    double* d_partial = nullptr;     // [kMaxChunks][9][T]
    int nchunk = 1;                  // far field: source chunks (grid y)
    int far_tpt = 1;                 // far field: targets per thread
    int self_pf[4] = {0, 0, 0, 0};   // self-interaction: Legendre prefetch batch per degree class (0: default)

    // graph mode: the launch sequence of ehd_layer_potentials recorded once
    // per argument set and replayed
    bool graph_on = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphKey {
        const void *f, *u, *s;
        void *so, *fo;
        unsigned kinds;
        int prec, tpt, nchunk;
        bool operator==(const GraphKey& o) const
        {
            return f == o.f && u == o.u && s == o.s && so == o.so && fo == o.fo && kinds == o.kinds &&
                   prec == o.prec && tpt == o.tpt && nchunk == o.nchunk;
        }
    } gkey{};
    hipStream_t ls = nullptr;        // stream the current evaluation launches on
    bool capturing = false;
    // overlap mode: the far field on its own stream, concurrent with the
    // self-interaction (forked after the densities, joined before combine)
    bool overlap = false;
    hipStream_t far_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // registers per lane (rounded to the allocation granule) and static LDS
    // bytes of each kernel as built, queried once per kernel
    struct KernRes { int vgpr, lds; };
    std::map<const void*, KernRes> kres;

    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
    }
    int2* d_rows_p = nullptr;        // rows of own grids
    int2* d_rows_f = nullptr;        // rows of far grids
    int nrows_p = 0, nrows_f = 0;
    int2* d_an_items = nullptr;
    int n_an_items = 0;

    // stage timing
    static constexpr int kStages = 4;
    static constexpr int kEv = kStages + 1 + 8;   // stage marks, then (start, end) per degree class
    std::vector<hipEvent_t> events;  // [nslots][kEv]
    std::vector<int> slot_used;
    std::vector<int> class_used;     // [nslots][4]
    int nslots = 0;
    long long ncalls = 0;

    void free_events()
    {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        events.clear();
        slot_used.clear();
        class_used.clear();
        nslots = 0;
    }
    void mark(int stage)
    {
        if (!nslots || capturing) return;
        const long long slot = ncalls % nslots;
        if (stage == 0)
            for (int c = 0; c < 4; ++c) class_used[slot * 4 + c] = 0;
        (void)hipEventRecord(events[slot * kEv + stage], stream);
    }
    void mark_class(int cls, int end)
    {
        if (!nslots || capturing) return;
        const long long slot = ncalls % nslots;
        (void)hipEventRecord(events[slot * kEv + kStages + 1 + 2 * cls + end], stream);
        class_used[slot * 4 + cls] = 1;
    }
    DropInfo* d_info_tmp = nullptr;  // per-field views for ehd_synthesize

    // nearly singular targets (ehd_set_near); its buffers live in near_allocs
    struct Near {
        double delta = 0.0, sc = 0.0;
        int m = 0, qc = 0;
        bool on = false;
        int npairs = 0, nfd = 0;         // pairs, drops with a check grid
        long long nf = 0;                // check-grid nodes
        std::vector<void*> allocs;
        NearPair* d_pairs = nullptr;
        double* d_legv = nullptr;        // Pbar, dPbar at the closest points
        DropInfo* d_fdrops = nullptr;    // check-grid views of the drops (leg_pf, soff)
        LegTab* d_flegs = nullptr;
        int2* d_frows = nullptr;
        int nfrows = 0;
        int* d_node_drop = nullptr;      // [nf] check-grid drop of each node
        long long* d_foff = nullptr;     // [nfd + 1] first node of each check grid
        int* d_fidx = nullptr;           // [nd] check grid of each drop (-1: none)
        double* d_frec = nullptr;        // [kRec64][nf]
        double* d_fsyn = nullptr;        // [9][nf]
        double* d_selfc = nullptr;       // [9][ncoef_total] projected self values
        double* d_lim = nullptr;         // [npairs][9]
        double* d_corr = nullptr;        // [npairs][9] each pair's correction of the output rows
        int ntgt = 0;                    // targets with at least one pair
        int* d_tlist = nullptr;          // [ntgt] those targets, increasing
        int* d_tstart = nullptr;         // [ntgt + 1] first pair of each (pairs are in target order)
        double* d_chk = nullptr;         // [npairs][kNearSplit][m+1][9]
        // check-grid tables per degree p, kept across shapes for (tab_qc, tab_gm)
        std::map<int, LegTab> tabs;
        std::vector<void*> tab_allocs;
        int tab_qc = -1, tab_gm = -1;
        void release()
        {
            for (void* a : allocs) (void)hipFree(a);
            allocs.clear();
            npairs = nfd = nfrows = ntgt = 0;
            nf = 0;
        }
        void release_tables()
        {
            for (void* a : tab_allocs) (void)hipFree(a);
            tab_allocs.clear();
            tabs.clear();
            tab_qc = tab_gm = -1;
        }
    } near;

    void free_all()
    {
        near.release();
        near.release_tables();
        near.on = false;
        for (void* a : allocs) (void)hipFree(a);
        allocs.clear();
        d_info = nullptr;
        d_legs = nullptr;
        d_wigs = nullptr;
        nd = 0;
    }
};

static std::string g_create_err = "no error";

#define EHD_FAIL(ctx, code, ...)                                              \
    do {                                                                      \
        char _b[512];                                                         \
        snprintf(_b, sizeof(_b), __VA_ARGS__);                                \
        (ctx)->err = _b;                                                      \
        return (code);                                                        \
    } while (0)

#define EHD_HIP(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t _e = (call);                                                              \
        if (_e != hipSuccess)                                                                \
            EHD_FAIL(ctx, EHD_E_HIP, "%s failed: %s", #call, hipGetErrorString(_e));         \
    } while (0)

template <typename T>
static int dev_alloc(ehd_ctx* ctx, T** out, size_t count)
{
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, sizeof(T) * count);
    if (e != hipSuccess) {
        ctx->err = std::string("hipMalloc failed: ") + hipGetErrorString(e);
        return EHD_E_NOMEM;
    }
    ctx->allocs.push_back(p);
    *out = (T*)p;
    return EHD_OK;
}

template <typename T>
static int upload(ehd_ctx* ctx, T** out, const std::vector<T>& h)
{
    int rc = dev_alloc(ctx, out, h.size());
    if (rc) return rc;
    if (!h.empty()) {
        hipError_t e = hipMemcpyAsync(*out, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice,
                                      ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            ctx->err = std::string("upload failed: ") + hipGetErrorString(e);
            return EHD_E_HIP;
        }
    }
    return EHD_OK;
}

static const int kClassP[4] = {16, 24, 32, 48};
static int degree_class(int p)
{
    for (int c = 0; c < 4; ++c)
        if (p <= kClassP[c]) return c;
    return -1;
}

static size_t self_lds_bytes(const ehd_ctx* ctx, const std::vector<int>& drops, int nf)
{
    // rotated coefficients first; afterwards the same memory holds the
    // Fourier blocks of one latitude block and each wave's node buffer
    size_t best = 0;
    for (int d : drops) {
        const DropInfo& D = ctx->info[d];
        const QuarterGrid g = quarter_grid(D.p, D.nlon_s, self_row0(D.p));
        const size_t coef = (size_t)nf * ncoef(D.p) * 16;
        const size_t work = ((size_t)kLatBlock * g.nks * 64 +
                             (size_t)SelfClass<16>::NW * (64 * ((nf + 6) | 1) + (D.p <= 32 ? 16 : 0)) +
                             (self_row0(D.p) ? (size_t)2 * kLatBlock * ((nf + 6) | 1) : 0)) * 8;
        best = std::max(best, std::max(coef, work));
    }
    return best;
}

// The self-interaction kernel of degree class PMAX for a field set and a
// Legendre prefetch batch (pf 0: the class default; other batches are built
// for the field set x, f, sigma only).
template <int PMAX, bool HF, bool HU, bool HS>
static const void* self_kernel_pf(int pf)
{
    using SC = SelfClass<PMAX>;
    if constexpr (HF && !HU && HS) {
        if (pf == SC::PF_ALT0) return (const void*)k_self<PMAX, HF, HU, HS, SC::PF_ALT0>;
        if (pf == SC::PF_ALT1) return (const void*)k_self<PMAX, HF, HU, HS, SC::PF_ALT1>;
    }
    return (const void*)k_self<PMAX, HF, HU, HS>;
}

// Launch of one degree class's self-interaction with the context's prefetch
// batch for the class (ehd_set_self_config), over the targets of the class.
template <int PMAX, bool HF, bool HU, bool HS>
static int launch_self_class(ehd_ctx* ctx, int cls, const double* f, const double* u, const double* s,
                             unsigned kinds)
{
    constexpr int NF = 3 + (HF ? 3 : 0) + (HU ? 3 : 0) + (HS ? 1 : 0);
    const int count = ctx->cls_off[cls + 1] - ctx->cls_off[cls];
    if (count == 0) return EHD_OK;
    const size_t lds = self_lds_bytes(ctx, ctx->cls_drops[cls], NF);
    const size_t lds_static = (size_t)SelfClass<PMAX>::NW * 9 * 8;   // reduction scratch
    if (lds + lds_static > (size_t)ctx->max_lds)
        EHD_FAIL(ctx, EHD_E_SHAPE, "self-interaction needs %zu bytes of LDS (limit %d)", lds, ctx->max_lds);
    const void* fn = self_kernel_pf<PMAX, HF, HU, HS>(ctx->self_pf[cls]);
    if (lds > 65536) EHD_HIP(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ctx->mark_class(cls, 0);
    const DropInfo* a0 = ctx->d_info;
    const LegTab* a1 = ctx->d_legs;
    const WigTab* a2 = ctx->d_wigs;
    const int* a3 = ctx->d_order + ctx->cls_off[cls];
    const int* a4 = ctx->d_tdrop;
    const double* a5 = ctx->d_x;
    const double *a9 = ctx->d_tx, *a10 = ctx->d_tn;
    long long a11 = ctx->T;
    double* a13 = ctx->d_raw;
    void* args[] = {(void*)&a0, (void*)&a1, (void*)&a2, (void*)&a3, (void*)&a4, (void*)&a5, (void*)&f, (void*)&u,
                    (void*)&s, (void*)&a9, (void*)&a10, (void*)&a11, (void*)&kinds, (void*)&a13};
    EHD_HIP(ctx, hipLaunchKernel(fn, dim3((unsigned)count), dim3(SelfClass<PMAX>::NT), args, lds, ctx->ls));
    ctx->mark_class(cls, 1);
    return EHD_OK;
}

// The degree classes in the mask (bit 3: p <= 48 .. bit 0: p <= 16), largest first.
template <bool HF, bool HU, bool HS>
static int launch_self(ehd_ctx* ctx, const double* f, const double* u, const double* s, unsigned kinds, unsigned cm)
{
    int rc = EHD_OK;
    if (!rc && (cm & 8u)) rc = launch_self_class<48, HF, HU, HS>(ctx, 3, f, u, s, kinds);
    if (!rc && (cm & 4u)) rc = launch_self_class<32, HF, HU, HS>(ctx, 2, f, u, s, kinds);
    if (!rc && (cm & 2u)) rc = launch_self_class<24, HF, HU, HS>(ctx, 1, f, u, s, kinds);
    if (!rc && (cm & 1u)) rc = launch_self_class<16, HF, HU, HS>(ctx, 0, f, u, s, kinds);
    return rc;
}

// The self-interaction kernel of degree class PMAX for the fields it holds
// and a prefetch batch.
template <int PMAX>
static const void* self_kernel(bool HF, bool HU, bool HS, int pf)
{
    if (HU) return self_kernel_pf<PMAX, false, true, false>(pf);
    if (HF && HS) return self_kernel_pf<PMAX, true, false, true>(pf);
    if (HF) return self_kernel_pf<PMAX, true, false, false>(pf);
    return self_kernel_pf<PMAX, false, false, true>(pf);
}
static const void* self_kernel_of_class(int cls, bool HF, bool HU, bool HS, int pf)
{
    return cls == 0 ? self_kernel<16>(HF, HU, HS, pf) : cls == 1 ? self_kernel<24>(HF, HU, HS, pf)
           : cls == 2 ? self_kernel<32>(HF, HU, HS, pf) : self_kernel<48>(HF, HU, HS, pf);
}

// FP64 far-field launchers, one per (targets per thread, kinds mask).
using Far64Launch = void (*)(dim3, hipStream_t, const double*, const double*, const int*, long long, const double*,
                             long long, const int2*, int, int, double*, int, int, int);
template <int TPT, unsigned KM>
static void launch_far64_km(dim3 grid, hipStream_t st, const double* tx, const double* tn, const int* tdrop,
                            long long T, const double* src, long long S, const int2* tile_info, int ntiles, int tpc,
                            double* partial, int nbx, int vb0, int vb1)
{
    hipLaunchKernelGGL((k_far64<TPT, KM>), grid, dim3(kThreads), 0, st, tx, tn, tdrop, T, src, S, tile_info, ntiles,
                       tpc, partial, nbx, vb0, vb1);
}
template <int TPT, std::size_t... I>
static const std::array<Far64Launch, 32>& far64_table_impl(std::index_sequence<I...>)
{
    static const std::array<Far64Launch, 32> t{{&launch_far64_km<TPT, (unsigned)I>...}};
    return t;
}
template <int TPT>
static const std::array<Far64Launch, 32>& far64_table()
{
    return far64_table_impl<TPT>(std::make_index_sequence<32>{});
}

// FP32 far-field launchers, one per (targets per thread, kinds mask).
using Far32Launch = void (*)(dim3, hipStream_t, const double*, const double*, const int*, long long, const float*,
                             long long, const int2*, const double*, int, int, double*, int, int, int);
template <int TPT, unsigned KM>
static void launch_far32_km(dim3 grid, hipStream_t st, const double* tx, const double* tn, const int* tdrop,
                            long long T, const float* src, long long S, const int2* tile_info, const double* centre,
                            int ntiles, int tpc, double* partial, int nbx, int vb0, int vb1)
{
    hipLaunchKernelGGL((k_far32<TPT, KM>), grid, dim3(kThreads), 0, st, tx, tn, tdrop, T, src, S, tile_info, centre,
                       ntiles, tpc, partial, nbx, vb0, vb1);
}
template <int TPT, std::size_t... I>
static const std::array<Far32Launch, 32>& far32_table_impl(std::index_sequence<I...>)
{
    static const std::array<Far32Launch, 32> t{{&launch_far32_km<TPT, (unsigned)I>...}};
    return t;
}
template <int TPT>
static const std::array<Far32Launch, 32>& far32_table()
{
    return far32_table_impl<TPT>(std::make_index_sequence<32>{});
}
// The FP32 far-field kernels themselves (resource queries).
template <int TPT, std::size_t... I>
static const std::array<const void*, 32>& far32_kernels_impl(std::index_sequence<I...>)
{
    static const std::array<const void*, 32> t{{(const void*)k_far32<TPT, (unsigned)I>...}};
    return t;
}
static const void* far32_kernel(int tpt, unsigned kinds)
{
    return (tpt == 2 ? far32_kernels_impl<2>(std::make_index_sequence<32>{})
                     : far32_kernels_impl<1>(std::make_index_sequence<32>{}))[kinds & EHD_ALL_KINDS];
}

// Accessors for the solvers (ctx_access.h).
hipStream_t ehd_ctx_stream(const ehd_ctx* ctx) { return ctx->stream; }
int ehd_ctx_device(const ehd_ctx* ctx) { return ctx->device; }
int ehd_ctx_ndrops(const ehd_ctx* ctx) { return ctx->nd; }
int ehd_ctx_drop_p(const ehd_ctx* ctx, int d) { return ctx->info[d].p; }
int ehd_ctx_graph_on(const ehd_ctx* ctx) { return ctx->graph_on ? 1 : 0; }
int ehd_ctx_fail(ehd_ctx* ctx, int code, const char* msg)
{
    ctx->err = msg;
    return code;
}

// --- nearly singular targets: host set-up ---------------------------------
template <typename T>
static int near_upload(ehd_ctx* ctx, T** out, const std::vector<T>& h, std::vector<void*>* owner = nullptr)
{
    void* p = nullptr;
    EHD_HIP(ctx, hipMalloc(&p, sizeof(T) * std::max<size_t>(h.size(), 1)));
    (owner ? owner : &ctx->near.allocs)->push_back(p);
    if (!h.empty())
        EHD_HIP(ctx, hipMemcpyAsync(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, ctx->stream));
    *out = (T*)p;
    return EHD_OK;
}

// A zeroed device buffer of n doubles owned by the near set-up.
static int near_zeros(ehd_ctx* ctx, double** out, size_t n)
{
    void* p = nullptr;
    EHD_HIP(ctx, hipMalloc(&p, sizeof(double) * std::max<size_t>(n, 1)));
    ctx->near.allocs.push_back(p);
    EHD_HIP(ctx, hipMemsetAsync(p, 0, sizeof(double) * std::max<size_t>(n, 1), ctx->stream));
    *out = (double*)p;
    return EHD_OK;
}

// x, dx/dtheta and dx/dphi of one drop's surface (3 packed fields) at (th, ph).
// The square-root factors of the orthonormal associated Legendre recurrence
// in theta (and of its ladder formula for d/dtheta) for one degree, so that a
// point costs no square roots; values agree bit for bit with the grid tables.
struct HostLeg {
    int p = -1;
    std::vector<double> diag, a, b, up, dn, row, P, dP, tg;
    explicit HostLeg(int p_) : p(p_)
    {
        const int pp = p + 1;
        diag.assign(pp + 1, 0.0);
        a.assign(ncoef(pp), 0.0);
        b.assign(ncoef(pp), 0.0);
        for (int m = 1; m <= pp; ++m) diag[m] = std::sqrt((2.0 * m + 1.0) / (2.0 * m));
        for (int m = 0; m <= pp; ++m)
            for (int n = m + 2; n <= pp; ++n) {
                a[tri(n, m)] = std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
                b[tri(n, m)] = std::sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
            }
        up.assign(ncoef(p), 0.0);
        dn.assign(ncoef(p), 0.0);
        for (int n = 0; n <= p; ++n)
            for (int m = 0; m <= n; ++m) {
                up[tri(n, m)] = (m + 1 <= n) ? std::sqrt((double)(n - m) * (n + m + 1)) : 0.0;
                dn[tri(n, m)] = m >= 1 ? std::sqrt((double)(n + m) * (n - m + 1)) : (n >= 1 ? -std::sqrt((double)n * (n + 1)) : 0.0);
            }
        row.assign(ncoef(pp), 0.0);
        P.assign(ncoef(p), 0.0);
        dP.assign(ncoef(p), 0.0);
        std::vector<double> w;
        ehd::gauss_legendre(p + 1, tg, w);
    }
    // P and dP/dtheta at cos(theta) = x
    void eval(double x)
    {
        const double s = std::sqrt((1.0 - x) * (1.0 + x));
        const int pp = p + 1;
        double dg = 1.0 / std::sqrt(4.0 * kPi);
        for (int m = 0; m <= pp; ++m) {
            if (m > 0) dg *= -diag[m] * s;
            row[tri(m, m)] = dg;
            if (m + 1 <= pp) row[tri(m + 1, m)] = std::sqrt(2.0 * m + 3.0) * x * dg;
            for (int n = m + 2; n <= pp; ++n) {
                const long k = tri(n, m);
                row[k] = a[k] * (x * row[tri(n - 1, m)] - b[k] * row[tri(n - 2, m)]);
            }
        }
        for (int n = 0; n <= p; ++n)
            for (int m = 0; m <= n; ++m) {
                const long k = tri(n, m);
                P[k] = row[k];
                const double u = (m + 1 <= n) ? up[k] * row[tri(n, m + 1)] : 0.0;
                const double d = (m >= 1) ? dn[k] * row[tri(n, m - 1)] : (n >= 1 ? dn[k] * row[tri(n, 1)] : 0.0);
                dP[k] = 0.5 * (u - d);
            }
    }
};

static void host_surface_point(HostLeg& L, const double* xc, double th, double ph, double x[3], double xt[3], double xp[3])
{
    const int p = L.p;
    L.eval(std::cos(th));
    const std::vector<double>&P = L.P, &dP = L.dP;
    const long nc = ncoef(p);
    for (int c = 0; c < 3; ++c) x[c] = xt[c] = xp[c] = 0.0;
    for (int m = 0; m <= p; ++m) {
        const double cm = std::cos(m * ph), sm = std::sin(m * ph), mult = m ? 2.0 : 1.0;
        for (int n = m; n <= p; ++n) {
            const long k = tri(n, m);
            for (int c = 0; c < 3; ++c) {
                const double cr = xc[2 * (c * nc + k)], ci = m ? xc[2 * (c * nc + k) + 1] : 0.0;
                const double re = cr * cm - ci * sm;
                x[c] += mult * re * P[k];
                xt[c] += mult * re * dP[k];
                xp[c] -= mult * m * (cr * sm + ci * cm) * P[k];
            }
        }
    }
}

// Near pairs of the current shapes, closest points, check grids.
static int near_build(ehd_ctx* ctx)
{
    ehd_ctx::Near& N = ctx->near;
    EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    N.release();
    if (!N.on) return EHD_OK;
    const long long T = ctx->T;
    std::vector<double> xh(3 * ctx->ncoef_total), tx(3 * T);
    EHD_HIP(ctx, hipMemcpyAsync(xh.data(), ctx->d_x, sizeof(double) * xh.size(), hipMemcpyDeviceToHost, ctx->stream));
    EHD_HIP(ctx, hipMemcpyAsync(tx.data(), ctx->d_tx, sizeof(double) * tx.size(), hipMemcpyDeviceToHost, ctx->stream));
    EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int nd = ctx->nd;
    // radius of each drop about its centre over its grid nodes
    std::vector<double> rho(nd, 0.0);
    std::vector<int> tdrop(T);
    for (int d = 0; d < nd; ++d) {
        const DropInfo& D = ctx->info[d];
        const long long n = (long long)(D.p + 1) * D.nlon_p;
        for (long long t = D.toff; t < D.toff + n; ++t) {
            tdrop[t] = d;
            double r2 = 0.0;
            for (int c = 0; c < 3; ++c) r2 += (tx[c * T + t] - D.c[c]) * (tx[c * T + t] - D.c[c]);
            rho[d] = std::max(rho[d], std::sqrt(r2));
        }
    }
    // chunks of 16 targets dealt round-robin to host threads (near targets
    // cluster), then the pairs put back in target order
    struct Part {
        std::vector<NearPair> pairs;
        std::vector<double> legv;
    };
    const int nth = (int)std::max(1LL, std::min<long long>({16LL, (long long)std::thread::hardware_concurrency(), T / 256}));
    std::vector<Part> parts(nth);
    auto search = [&](int w) {
        Part& R = parts[w];
        std::map<int, HostLeg> hleg;
        for (long long t = 0; t < T; ++t) {
            if ((t / 16) % nth != w) continue;
            const double x0[3] = {tx[t], tx[T + t], tx[2 * T + t]};
            for (int j = 0; j < nd; ++j) {
                if (j == tdrop[t]) continue;
                const DropInfo& D = ctx->info[j];
                double d0 = 0.0;
                for (int c = 0; c < 3; ++c) d0 += (x0[c] - D.c[c]) * (x0[c] - D.c[c]);
                if (std::sqrt(d0) > 1.2 * rho[j] + N.delta) continue;
                // nearest grid node of drop j, then damped Gauss-Newton in (theta, phi)
                const long long n = (long long)(D.p + 1) * D.nlon_p;
                long long best = D.toff;
                double bd = 1e300;
                for (long long q = D.toff; q < D.toff + n; ++q) {
                    double e = 0.0;
                    for (int c = 0; c < 3; ++c) e += (tx[c * T + q] - x0[c]) * (tx[c * T + q] - x0[c]);
                    if (e < bd) { bd = e; best = q; }
                }
                // the surface is within half a node spacing (about pi rho / (p + 1)
                // along a parallel, less along a meridian) of its nearest node
                if (std::sqrt(bd) > N.delta + kPi * rho[j] / (D.p + 1)) continue;
                HostLeg& HL = hleg.try_emplace(D.p, D.p).first->second;
                const std::vector<double>& tg = HL.tg;
                const long long loc = best - D.toff;
                double th = std::acos(tg[loc / D.nlon_p]), ph = 2.0 * kPi * (double)(loc % D.nlon_p) / D.nlon_p;
                const double* xc = xh.data() + 3 * D.coff;
                double x[3], xt[3], xp[3];
                for (int it = 0; it < 60; ++it) {
                    host_surface_point(HL, xc, th, ph, x, xt, xp);
                    double r[3], A00 = 0, A01 = 0, A11 = 0, g0 = 0, g1 = 0;
                    for (int c = 0; c < 3; ++c) {
                        r[c] = x[c] - x0[c];
                        A00 += xt[c] * xt[c]; A01 += xt[c] * xp[c]; A11 += xp[c] * xp[c];
                        g0 += xt[c] * r[c]; g1 += xp[c] * r[c];
                    }
                    const double mu = 1e-14 * (A00 + A11);
                    A00 += mu; A11 += mu;
                    const double det = A00 * A11 - A01 * A01;
                    const double d_th = -(A11 * g0 - A01 * g1) / det, d_ph = -(A00 * g1 - A01 * g0) / det;
                    th = std::min(kPi - 1e-9, std::max(1e-9, th + d_th));
                    ph += d_ph;
                    if (std::fabs(d_th) + std::fabs(d_ph) < 1e-15) break;
                }
                host_surface_point(HL, xc, th, ph, x, xt, xp);
                const std::vector<double>&P = HL.P, &dP = HL.dP;
                double dist = 0.0;
                for (int c = 0; c < 3; ++c) dist += (x0[c] - x[c]) * (x0[c] - x[c]);
                dist = std::sqrt(dist);
                if (!(dist < N.delta) || dist < 1e-12) continue;
                NearPair pr{};
                pr.t = (int)t;
                pr.j = j;
                pr.th = th;
                pr.ph = ph;
                const double cx = xt[1] * xp[2] - xt[2] * xp[1], cy = xt[2] * xp[0] - xt[0] * xp[2],
                             cz = xt[0] * xp[1] - xt[1] * xp[0];
                const double cn = std::sqrt(cx * cx + cy * cy + cz * cz);
                const double nrm[3] = {cx / cn, cy / cn, cz / cn};
                for (int c = 0; c < 3; ++c) {
                    pr.y[c] = x[c];
                    pr.ny[c] = nrm[c];
                    pr.xt[c] = xt[c];
                    pr.xp[c] = xp[c];
                    pr.nu[c] = (x0[c] - x[c]) / dist;
                }
                pr.st = dist;
                pr.legoff = (long long)R.legv.size();
                R.legv.insert(R.legv.end(), P.begin(), P.end());
                R.legv.insert(R.legv.end(), dP.begin(), dP.end());
                R.pairs.push_back(pr);
            }
        }
    };
    std::atomic<bool> failed{false};
    auto run = [&](int w) {
        try {
            search(w);
        } catch (...) {   // host allocation: reported below, never across the ABI
            failed = true;
        }
    };
    std::vector<std::thread> workers;
    for (int w = 1; w < nth; ++w) {
        try {
            workers.emplace_back(run, w);
        } catch (...) {   // no thread to be had: this one takes the part
            run(w);
        }
    }
    run(0);
    for (std::thread& th : workers) th.join();
    if (failed) EHD_FAIL(ctx, EHD_E_NOMEM, "near set-up: host allocation failed");
    std::vector<std::pair<int, int>> order;   // (part, index) by target
    for (int w = 0; w < nth; ++w)
        for (int i = 0; i < (int)parts[w].pairs.size(); ++i) order.emplace_back(w, i);
    std::stable_sort(order.begin(), order.end(), [&](const std::pair<int, int>& a, const std::pair<int, int>& b) {
        return parts[a.first].pairs[a.second].t < parts[b.first].pairs[b.second].t;
    });
    std::vector<NearPair> pairs;
    std::vector<double> legv;
    for (const std::pair<int, int>& o : order) {
        NearPair pr = parts[o.first].pairs[o.second];
        const double* src = parts[o.first].legv.data() + pr.legoff;
        pr.legoff = (long long)legv.size();
        legv.insert(legv.end(), src, src + 2 * ncoef(ctx->info[pr.j].p));
        pairs.push_back(pr);
    }
    N.npairs = (int)pairs.size();
    if (!N.npairs) return EHD_OK;
    // the corrected targets and the first of each one's (consecutive) pairs
    std::vector<int> tlist, tstart;
    for (int i = 0; i < N.npairs; ++i)
        if (i == 0 || pairs[i].t != pairs[i - 1].t) {
            tlist.push_back(pairs[i].t);
            tstart.push_back(i);
        }
    tstart.push_back(N.npairs);
    N.ntgt = (int)tlist.size();
    // check grids (degree qc) of the drops with pairs
    std::vector<int> fidx(nd, -1);
    for (const NearPair& pr : pairs) fidx[pr.j] = 0;
    std::vector<DropInfo> fd;
    std::vector<LegTab> fl;
    std::vector<long long> foff{0};
    std::vector<int2> frows;
    std::vector<int> node_drop;
    std::map<int, int> legid;
    if (N.tab_qc != N.qc || N.tab_gm != ctx->grid_mode) {
        N.release_tables();
        N.tab_qc = N.qc;
        N.tab_gm = ctx->grid_mode;
    }
    for (int j = 0; j < nd; ++j) {
        if (fidx[j] < 0) continue;
        fidx[j] = (int)fd.size();
        DropInfo D = ctx->info[j];
        const int Q = N.qc, nl = nlon_of(Q, ctx->grid_mode);
        auto it = legid.find(D.p);
        if (it == legid.end() && N.tabs.count(D.p)) {
            fl.push_back(N.tabs[D.p]);
            it = legid.emplace(D.p, (int)fl.size() - 1).first;
        }
        if (it == legid.end()) {
            std::vector<double> t, w, P, dP;
            ehd::gauss_legendre(Q + 1, t, w);
            ehd::legendre_tables(D.p, t, P, dP);
            std::vector<double> wq(Q + 1), rs(Q + 1), trig((size_t)nl * (D.p + 1) * 2);
            for (int i = 0; i <= Q; ++i) {
                wq[i] = 2.0 * kPi / nl * w[i];
                rs[i] = 1.0 / std::sqrt((1.0 - t[i]) * (1.0 + t[i]));
            }
            for (int l = 0; l < nl; ++l)
                for (int m = 0; m <= D.p; ++m) {
                    const double a = 2.0 * kPi * (double)((long)m * l % nl) / nl;
                    trig[((size_t)l * (D.p + 1) + m) * 2] = std::cos(a);
                    trig[((size_t)l * (D.p + 1) + m) * 2 + 1] = std::sin(a);
                }
            LegTab L{};
            double* dp;
            int rc;
            if ((rc = near_upload(ctx, &dp, P, &N.tab_allocs))) return rc;
            L.P = dp;
            if ((rc = near_upload(ctx, &dp, dP, &N.tab_allocs))) return rc;
            L.dP = dp;
            if ((rc = near_upload(ctx, &dp, wq, &N.tab_allocs))) return rc;
            L.wq = dp;
            if ((rc = near_upload(ctx, &dp, rs, &N.tab_allocs))) return rc;
            L.rsin = dp;
            if ((rc = near_upload(ctx, &dp, t, &N.tab_allocs))) return rc;
            L.cth = dp;
            if ((rc = near_upload(ctx, &dp, trig, &N.tab_allocs))) return rc;
            L.trig = dp;
            L.p = D.p;
            L.Q = Q;
            L.nlon = nl;
            fl.push_back(L);
            N.tabs[D.p] = L;
            it = legid.emplace(D.p, (int)fl.size() - 1).first;
        }
        D.leg_pf = it->second;
        D.qf = Q;
        D.nlon_f = nl;
        D.soff = foff.back();
        D.ns = (long long)(Q + 1) * nl;
        for (int i = 0; i <= Q; ++i) frows.push_back(make_int2((int)fd.size(), i));
        for (long long q = 0; q < D.ns; ++q) node_drop.push_back((int)fd.size());
        foff.push_back(foff.back() + D.ns);
        fd.push_back(D);
    }
    N.nfd = (int)fd.size();
    N.nf = foff.back();
    N.nfrows = (int)frows.size();
    int rc;
    if ((rc = near_upload(ctx, &N.d_pairs, pairs)) || (rc = near_upload(ctx, &N.d_legv, legv)) ||
        (rc = near_upload(ctx, &N.d_fdrops, fd)) || (rc = near_upload(ctx, &N.d_flegs, fl)) ||
        (rc = near_upload(ctx, &N.d_frows, frows)) || (rc = near_upload(ctx, &N.d_node_drop, node_drop)) ||
        (rc = near_upload(ctx, &N.d_foff, foff)) || (rc = near_upload(ctx, &N.d_fidx, fidx)) ||
        (rc = near_upload(ctx, &N.d_tlist, tlist)) || (rc = near_upload(ctx, &N.d_tstart, tstart)))
        return rc;
    if ((rc = near_zeros(ctx, &N.d_frec, (size_t)kRec64 * N.nf)) || (rc = near_zeros(ctx, &N.d_fsyn, (size_t)9 * N.nf)) ||
        (rc = near_zeros(ctx, &N.d_selfc, (size_t)9 * ctx->ncoef_total)) ||
        (rc = near_zeros(ctx, &N.d_lim, (size_t)9 * N.npairs)) ||
        (rc = near_zeros(ctx, &N.d_corr, (size_t)9 * N.npairs)) ||
        (rc = near_zeros(ctx, &N.d_chk, (size_t)9 * (N.m + 1) * kNearSplit * N.npairs)))
        return rc;
    // check-grid geometry
    hipLaunchKernelGGL((k_synth<3, true>), dim3(N.nfrows), dim3(kThreads), 0, ctx->stream, N.d_fdrops, N.d_flegs, 1,
                       N.d_frows, ctx->d_x, N.d_fsyn, N.nf);
    hipLaunchKernelGGL(k_fine_geom, dim3((N.nf + 255) / 256), dim3(256), 0, ctx->stream, N.d_fdrops, N.d_flegs,
                       N.d_node_drop, N.d_fsyn, N.nf, N.d_frec);
    EHD_HIP(ctx, hipGetLastError());
    EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return EHD_OK;
}

// Device work of the nearly singular correction of one evaluation, after
// the outputs are combined (out: the far part, or the sum).
static int near_enqueue(ehd_ctx* ctx, const double* fcoef_d, const double* ucoef_d, const double* sigcoef_d,
                        const RowMap& rows, double* out)
{
    ehd_ctx::Near& N = ctx->near;
    const long long nf = N.nf;
    double* synf = fcoef_d ? N.d_fsyn : nullptr;
    double* synu = ucoef_d ? N.d_fsyn + 3 * nf : nullptr;
    double* syns = sigcoef_d ? N.d_fsyn + 6 * nf : nullptr;
    if (synf)
        hipLaunchKernelGGL((k_synth<3, false>), dim3(N.nfrows), dim3(kThreads), 0, ctx->ls, N.d_fdrops, N.d_flegs, 1,
                           N.d_frows, fcoef_d, synf, nf);
    if (synu)
        hipLaunchKernelGGL((k_synth<3, false>), dim3(N.nfrows), dim3(kThreads), 0, ctx->ls, N.d_fdrops, N.d_flegs, 1,
                           N.d_frows, ucoef_d, synu, nf);
    if (syns)
        hipLaunchKernelGGL((k_synth<1, false>), dim3(N.nfrows), dim3(kThreads), 0, ctx->ls, N.d_fdrops, N.d_flegs, 1,
                           N.d_frows, sigcoef_d, syns, nf);
    hipLaunchKernelGGL(k_fine_dens, dim3((nf + 255) / 256), dim3(256), 0, ctx->ls, synf, synu, syns, nf, N.d_frec);
    hipLaunchKernelGGL(k_analyze, dim3(ctx->n_an_items), dim3(kThreads), 0, ctx->ls, ctx->d_info, ctx->d_legs,
                       ctx->d_an_items, 9, ctx->d_raw, ctx->T, N.d_selfc);
    const double* uc = ucoef_d ? ucoef_d : fcoef_d;
    hipLaunchKernelGGL(k_near_limit, dim3(N.npairs), dim3(kThreads), 0, ctx->ls, N.d_pairs, ctx->d_info, N.d_legv,
                       N.d_selfc, uc ? uc : N.d_selfc, sigcoef_d ? sigcoef_d : N.d_selfc, ctx->d_tn, ctx->T, N.d_lim);
    hipLaunchKernelGGL(k_near_check, dim3(N.npairs, kNearSplit), dim3(kThreads), 0, ctx->ls, N.d_pairs, N.m, N.sc,
                       N.d_frec, nf, N.d_foff, N.d_fidx, ctx->d_tn, ctx->T, N.d_chk);
    hipLaunchKernelGGL(k_near_plain, dim3(N.npairs), dim3(kThreads), 0, ctx->ls, N.d_pairs, N.m, ctx->d_src64,
                       ctx->Spad, ctx->d_info, ctx->d_tx, ctx->d_tn, ctx->T, N.d_chk);
    hipLaunchKernelGGL(k_near_apply, dim3(N.npairs), dim3(128), 0, ctx->ls, N.d_pairs, N.m, N.sc, N.d_lim, N.d_chk,
                       rows, N.d_corr);
    const long long ng = (long long)N.ntgt * rows.n;
    hipLaunchKernelGGL(k_near_gather, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, ctx->ls, N.d_tstart,
                       N.d_tlist, N.ntgt, N.d_corr, rows, ctx->T, out);
    EHD_HIP(ctx, hipGetLastError());
    return EHD_OK;
}

extern "C" {

int ehd_create(ehd_ctx** out, int device, void* stream)
{
    if (!out) { g_create_err = "out is NULL"; return EHD_E_ARG; }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        g_create_err = "no HIP device";
        return EHD_E_HIP;
    }
    if (device < 0 || device >= ndev) { g_create_err = "device index out of range"; return EHD_E_ARG; }
    if (hipSetDevice(device) != hipSuccess) { g_create_err = "hipSetDevice failed"; return EHD_E_HIP; }
    ehd_ctx* c = new ehd_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
        lds > 0)
        c->max_lds = lds;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        c->ncu = ncu;
    *out = c;
    return EHD_OK;
}

void ehd_destroy(ehd_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    ctx->drop_graph();
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->far_stream) (void)hipStreamDestroy(ctx->far_stream);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    ctx->free_all();
    ctx->free_events();
    delete ctx;
}

const char* ehd_last_error(const ehd_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int ehd_grid_dims(int P, int grid_mode, int* nlat, int* nlon)
{
    if (P < 1 || P > EHD_MAX_Q || (grid_mode != 0 && grid_mode != 1) || !nlat || !nlon) return EHD_E_ARG;
    *nlat = P + 1;
    *nlon = nlon_of(P, grid_mode);
    return EHD_OK;
}

int ehd_wigner_d(int n, double beta, double* out)
{
    if (n < 0 || n > 200 || !out) return EHD_E_ARG;
    std::vector<double> d;
    ehd::wigner_d(n, beta, d);
    std::memcpy(out, d.data(), sizeof(double) * d.size());
    return EHD_OK;
}

// Drop centres (the degree-0 coefficients of x over sqrt(4 pi)) into
// ctx->info, read from the context's copy of x.
static int read_centres(ehd_ctx* ctx)
{
    std::vector<double> c00(3 * ctx->nd);
    for (int d = 0; d < ctx->nd; ++d)
        for (int c = 0; c < 3; ++c)
            EHD_HIP(ctx, hipMemcpyAsync(&c00[3 * d + c],
                                        ctx->d_x + 3 * ctx->info[d].coff +
                                            (long long)c * (ctx->info[d].p + 1) * (ctx->info[d].p + 2),
                                        sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int d = 0; d < ctx->nd; ++d)
        for (int c = 0; c < 3; ++c) ctx->info[d].c[c] = c00[3 * d + c] / std::sqrt(4.0 * kPi);
    return EHD_OK;
}

// Target geometry on the own grids and far-source geometry on the far grids
// from the context's copy of x.  Synchronous.
static int build_geometry(ehd_ctx* ctx)
{
    const long long T = ctx->T, S = ctx->Spad, vs = ctx->syn_stride;
    hipLaunchKernelGGL((k_synth<3, true>), dim3(ctx->nrows_p), dim3(kThreads), 0, ctx->stream,
                       ctx->d_info, ctx->d_legs, 0, ctx->d_rows_p, ctx->d_x, ctx->d_syn, vs);
    hipLaunchKernelGGL(k_geom_targets, dim3((T + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_syn, vs, T,
                       ctx->d_tx, ctx->d_tn);
    hipLaunchKernelGGL((k_synth<3, true>), dim3(ctx->nrows_f), dim3(kThreads), 0, ctx->stream,
                       ctx->d_info, ctx->d_legs, 1, ctx->d_rows_f, ctx->d_x, ctx->d_syn, vs);
    hipLaunchKernelGGL(k_geom_sources, dim3((S + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_info,
                       ctx->d_legs, ctx->d_slot_drop, ctx->d_syn, vs, S, ctx->d_src64, ctx->d_src32);
    hipLaunchKernelGGL(k_drop_radius, dim3(ctx->nd), dim3(kThreads), 0, ctx->stream, ctx->d_info, ctx->d_src64, S,
                       ctx->d_centre);
    EHD_HIP(ctx, hipGetLastError());
    EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return EHD_OK;
}

int ehd_set_drops(ehd_ctx* ctx, int ndrops, const int* p_h, const int* q_self_h, const int* q_far_h,
                  int grid_mode, const double* xcoef_d)
{
    if (!ctx) return EHD_E_ARG;
    if (ndrops < 1 || !p_h || !q_self_h || !q_far_h || !xcoef_d)
        EHD_FAIL(ctx, EHD_E_ARG, "ndrops must be >= 1 and all pointers non-NULL");
    if (grid_mode != 0 && grid_mode != 1) EHD_FAIL(ctx, EHD_E_ARG, "grid_mode must be 0 or 1");
    if (((uintptr_t)xcoef_d) % 8) EHD_FAIL(ctx, EHD_E_ARG, "xcoef_d must be 8-byte aligned");
    for (int d = 0; d < ndrops; ++d) {
        if (p_h[d] < 1 || p_h[d] > EHD_MAX_P)
            EHD_FAIL(ctx, EHD_E_SHAPE, "drop %d: p = %d outside [1, %d]", d, p_h[d], EHD_MAX_P);
        if (q_self_h[d] < p_h[d] || q_self_h[d] > EHD_MAX_Q || q_far_h[d] < p_h[d] || q_far_h[d] > EHD_MAX_Q)
            EHD_FAIL(ctx, EHD_E_SHAPE, "drop %d: q_self = %d, q_far = %d must lie in [p, %d]", d,
                     q_self_h[d], q_far_h[d], EHD_MAX_Q);
        if (grid_mode == 1 && p_h[d] < 2)
            EHD_FAIL(ctx, EHD_E_SHAPE, "grid_mode 1 needs p >= 2");
        if (nlon_of(q_self_h[d], grid_mode) > 256)
            EHD_FAIL(ctx, EHD_E_SHAPE, "drop %d: q_self = %d gives more than 256 longitudes on the rotated grid",
                     d, q_self_h[d]);
    }
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    if (ctx->stream) EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->drop_graph();
    ctx->free_all();
    int rc;
    ctx->nd = ndrops;
    ctx->grid_mode = grid_mode;
    ctx->p.assign(p_h, p_h + ndrops);
    ctx->qs.assign(q_self_h, q_self_h + ndrops);
    ctx->qf.assign(q_far_h, q_far_h + ndrops);

    // --- quadrature tables per distinct (p, Q) pair, rotation tables per p
    std::map<std::pair<int, int>, int> legid;
    std::map<int, int> wigid;
    std::vector<LegTab> legs;
    std::vector<WigTab> wigs;
    auto want_leg = [&](int pp, int Q, bool singular) -> int {
        auto key = std::make_pair(pp, Q * 2 + (singular ? 1 : 0));
        auto it = legid.find(key);
        if (it != legid.end()) return it->second;
        std::vector<double> t, w, P, dP, msum;
        ehd::gauss_legendre(Q + 1, t, w);
        ehd::legendre_tables(pp, t, P, dP);
        const int nl = nlon_of(Q, grid_mode);
        std::vector<double> wq(Q + 1), ws(Q + 1), rs(Q + 1), trig((size_t)nl * (pp + 1) * 2);
        ehd::singular_factor(Q, t, msum);
        for (int i = 0; i <= Q; ++i) {
            wq[i] = 2.0 * kPi / nl * w[i];
            ws[i] = wq[i] * msum[i];
            rs[i] = 1.0 / std::sqrt((1.0 - t[i]) * (1.0 + t[i]));
        }
        for (int l = 0; l < nl; ++l)
            for (int m = 0; m <= pp; ++m) {
                const double a = 2.0 * kPi * (double)((long)m * l % nl) / nl;
                trig[((size_t)l * (pp + 1) + m) * 2] = std::cos(a);
                trig[((size_t)l * (pp + 1) + m) * 2 + 1] = std::sin(a);
            }
        // MFMA A fragments of the quarter-period cos/sin tables (singular
        // grids): lane holds A[row l = l0 + 16 t + lane%16][term 4 ks + lane/16] of the
        // term groups EC (cos m, m = 0, 2, ..), ES (sin m, m = 2, 4, ..),
        // OC (cos m, m = 1, 3, ..), OS (sin m, m = 1, 3, ..), one after the other.
        std::vector<double> afrag;
        if (singular) {
            const QuarterGrid g = quarter_grid(pp, nl, self_row0(pp));
            afrag.assign((size_t)g.nT * g.nks * 64, 0.0);
            const int terms[4] = {pp / 2 + 1, pp / 2, (pp + 1) / 2, (pp + 1) / 2};
            for (int t = 0; t < g.nT; ++t)
                for (int grp = 0; grp < 4; ++grp)
                    for (int ks = 0; ks < g.nk[grp]; ++ks)
                        for (int lane = 0; lane < 64; ++lane) {
                            const int l = g.l0 + 16 * t + (lane & 15), term = 4 * ks + (lane >> 4);
                            if (l > g.H / 2 || term >= terms[grp]) continue;
                            const int m = grp == 0 ? 2 * term : grp == 1 ? 2 * term + 2 : 2 * term + 1;
                            const bool is_cos = grp == 0 || grp == 2;
                            const double a = 2.0 * kPi * (double)((long)m * l % nl) / nl;
                            afrag[((size_t)t * g.nks + g.base[grp] / 4 + ks) * 64 + lane] =
                                is_cos ? std::cos(a) : std::sin(a);
                        }
        }
        LegTab L{};
        double* dptr;
        if (singular) {
            if (upload(ctx, &dptr, afrag)) return -1;
            L.afrag = dptr;
        }
        if (upload(ctx, &dptr, P)) return -1;
        L.P = dptr;
        if (upload(ctx, &dptr, dP)) return -1;
        L.dP = dptr;
        if (upload(ctx, &dptr, wq)) return -1;
        L.wq = dptr;
        if (upload(ctx, &dptr, ws)) return -1;
        L.wsing = dptr;
        if (upload(ctx, &dptr, rs)) return -1;
        L.rsin = dptr;
        if (upload(ctx, &dptr, t)) return -1;
        L.cth = dptr;
        if (upload(ctx, &dptr, trig)) return -1;
        L.trig = dptr;
        if (singular) {
            // Legendre A fragments, per latitude block and per wave: the
            // k-steps of the wave's degree columns (snake order, increasing
            // m) back to back, zero-padded to the class's maximum; lane holds
            // row lane%16 (Pbar at latitudes 0..7 of the block, then
            // dPbar/dtheta), degree n = m + 4 ks + lane/16.
            const long ncp = ncoef(pp);
            const int nw = SelfClass<16>::NW, kw = self_kw(pp);
            const int nblk = (Q + 1 + kLatBlock - 1) / kLatBlock;
            std::vector<double> lf((size_t)nblk * nw * kw * 64, 0.0);
            for (int bb = 0; bb < nblk; ++bb)
                for (int w = 0; w < nw; ++w) {
                    int t = 0;
                    for (int m = 0; m <= pp; ++m) {
                        if (snake_wave(m, nw) != w) continue;
                        for (int ks = 0; ks < (pp + 1 - m + 3) / 4; ++ks, ++t)
                            for (int lane = 0; lane < 64; ++lane) {
                                const int row = lane & 15, n = m + 4 * ks + (lane >> 4);
                                const int lat = bb * kLatBlock + (row & 7);
                                if (lat > Q || n > pp) continue;
                                const std::vector<double>& tab = (row < 8) ? P : dP;
                                lf[(((size_t)bb * nw + w) * kw + t) * 64 + lane] = tab[(size_t)lat * ncp + tri(n, m)];
                            }
                    }
                    if (t > kw) return -1;
                }
            if (upload(ctx, &dptr, lf)) return -1;
            L.lfrag = dptr;
        }
        L.p = pp;
        L.Q = Q;
        L.nlon = nl;
        legs.push_back(L);
        legid[key] = (int)legs.size() - 1;
        return (int)legs.size() - 1;
    };
    auto want_wig = [&](int pp) -> int {
        auto it = wigid.find(pp);
        if (it != wigid.end()) return it->second;
        std::vector<double> t, w;
        ehd::gauss_legendre(pp + 1, t, w);
        const long wb = ehd::wig_block(pp);
        std::vector<double> A((size_t)(pp + 1) * wb), B((size_t)(pp + 1) * wb);
        for (int j = 0; j <= pp; ++j) {
            const double beta = std::atan2(std::sqrt((1.0 - t[j]) * (1.0 + t[j])), t[j]);
            ehd::rotation_blocks(pp, beta, A.data() + (size_t)j * wb, B.data() + (size_t)j * wb);
        }
        WigTab Wt{};
        double* dptr;
        if (upload(ctx, &dptr, A)) return -1;
        Wt.A = dptr;
        if (upload(ctx, &dptr, B)) return -1;
        Wt.B = dptr;
        Wt.p = pp;
        wigs.push_back(Wt);
        wigid[pp] = (int)wigs.size() - 1;
        return (int)wigs.size() - 1;
    };

    // --- per-drop layout
    ctx->info.assign(ndrops, DropInfo{});
    long long coff = 0, toff = 0, soff = 0;
    for (int d = 0; d < ndrops; ++d) {
        DropInfo& D = ctx->info[d];
        D.p = p_h[d];
        D.qs = q_self_h[d];
        D.qf = q_far_h[d];
        D.nlon_p = nlon_of(D.p, grid_mode);
        D.nlon_s = nlon_of(D.qs, grid_mode);
        D.nlon_f = nlon_of(D.qf, grid_mode);
        D.leg_pp = want_leg(D.p, D.p, false);
        D.leg_ps = want_leg(D.p, D.qs, true);
        D.leg_pf = want_leg(D.p, D.qf, false);
        D.wig = want_wig(D.p);
        if (D.leg_pp < 0 || D.leg_ps < 0 || D.leg_pf < 0 || D.wig < 0) return EHD_E_NOMEM;
        D.coff = coff;
        D.toff = toff;
        D.soff = soff;
        D.ns = (long long)(D.qf + 1) * D.nlon_f;
        coff += (long long)(D.p + 1) * (D.p + 2);
        toff += (long long)(D.p + 1) * D.nlon_p;
        soff += (D.ns + kTile - 1) / kTile * kTile;
    }
    ctx->ncoef_total = coff;
    ctx->T = toff;
    ctx->Spad = soff;
    ctx->ntiles = (int)(soff / kTile);
    if ((rc = upload(ctx, &ctx->d_legs, legs))) return rc;
    if ((rc = upload(ctx, &ctx->d_wigs, wigs))) return rc;

    // own copy of x, centres from the degree-0 coefficients
    if ((rc = dev_alloc(ctx, &ctx->d_x, 3 * coff))) return rc;
    EHD_HIP(ctx, hipMemcpyAsync(ctx->d_x, xcoef_d, sizeof(double) * 3 * coff, hipMemcpyDeviceToDevice,
                                ctx->stream));
    if ((rc = read_centres(ctx))) return rc;
    {
        std::vector<double> cen(4 * ndrops, 0.0);          // radii: build_geometry
        for (int d = 0; d < ndrops; ++d)
            for (int c = 0; c < 3; ++c) cen[4 * d + c] = ctx->info[d].c[c];
        if ((rc = upload(ctx, &ctx->d_centre, cen))) return rc;
    }
    if ((rc = upload(ctx, &ctx->d_info, ctx->info))) return rc;

    // index tables
    std::vector<int> tdrop(ctx->T), slot_drop(ctx->Spad);
    std::vector<int2> tile_info(ctx->ntiles);
    std::vector<int2> rows_p, rows_f, an_items;
    for (int d = 0; d < ndrops; ++d) {
        const DropInfo& D = ctx->info[d];
        for (long long t = 0; t < (long long)(D.p + 1) * D.nlon_p; ++t) tdrop[D.toff + t] = d;
        const long long padded = (D.ns + kTile - 1) / kTile * kTile;
        for (long long s = 0; s < padded; ++s) slot_drop[D.soff + s] = d;
        // the far-field kernels sum a tile's sources in fours; the padding
        // slots past a drop's last source are skipped
        for (long long tl = 0; tl < padded / kTile; ++tl)
            tile_info[D.soff / kTile + tl] =
                make_int2(d, (int)((std::min<long long>(kTile, D.ns - tl * kTile) + 3) / 4 * 4));
        for (int i = 0; i <= D.p; ++i) rows_p.push_back(make_int2(d, i));
        for (int i = 0; i <= D.qf; ++i) rows_f.push_back(make_int2(d, i));
        for (int k = 0; k < ncoef(D.p); ++k) an_items.push_back(make_int2(d, k));
    }
    // self work order: by degree class (largest first), inside a class the
    // most expensive drops first
    std::vector<int> dorder(ndrops);
    for (int d = 0; d < ndrops; ++d) dorder[d] = d;
    std::stable_sort(dorder.begin(), dorder.end(), [&](int a, int b) {
        const DropInfo &A = ctx->info[a], &B = ctx->info[b];
        const double ca = (double)(A.qs + 1) * A.nlon_s * (A.p + 1), cb = (double)(B.qs + 1) * B.nlon_s * (B.p + 1);
        return ca > cb;
    });
    ctx->self_order_h.clear();
    for (int c = 0; c < 4; ++c) ctx->cls_drops[c].clear();
    for (int cls = 0; cls < 4; ++cls) {
        ctx->cls_off[cls] = (int)ctx->self_order_h.size();
        for (int d : dorder) {
            const DropInfo& D = ctx->info[d];
            if (degree_class(D.p) != cls) continue;
            ctx->cls_drops[cls].push_back(d);
            for (long long t = 0; t < (long long)(D.p + 1) * D.nlon_p; ++t)
                ctx->self_order_h.push_back((int)(D.toff + t));
        }
    }
    ctx->cls_off[4] = (int)ctx->self_order_h.size();
    if ((rc = upload(ctx, &ctx->d_tdrop, tdrop))) return rc;
    if ((rc = upload(ctx, &ctx->d_slot_drop, slot_drop))) return rc;
    if ((rc = upload(ctx, &ctx->d_tile_info, tile_info))) return rc;
    if ((rc = upload(ctx, &ctx->d_rows_p, rows_p))) return rc;
    if ((rc = upload(ctx, &ctx->d_rows_f, rows_f))) return rc;
    if ((rc = upload(ctx, &ctx->d_an_items, an_items))) return rc;
    if ((rc = upload(ctx, &ctx->d_order, ctx->self_order_h))) return rc;
    ctx->nrows_p = (int)rows_p.size();
    ctx->nrows_f = (int)rows_f.size();
    ctx->n_an_items = (int)an_items.size();

    // work buffers
    const long long T = ctx->T, S = ctx->Spad;
    ctx->syn_stride = std::max(T, S);
    if ((rc = dev_alloc(ctx, &ctx->d_syn, 16 * ctx->syn_stride))) return rc;
    if ((rc = dev_alloc(ctx, &ctx->d_tx, 3 * T))) return rc;
    if ((rc = dev_alloc(ctx, &ctx->d_tn, 3 * T))) return rc;
    if ((rc = dev_alloc(ctx, &ctx->d_src64, (size_t)kRec64 * S))) return rc;
    if ((rc = dev_alloc(ctx, &ctx->d_src32, (size_t)kRec32 * S))) return rc;
    if ((rc = dev_alloc(ctx, &ctx->d_raw, 9 * T))) return rc;
    const long long tblocks = (T + kThreads - 1) / kThreads;
    ctx->far_tpt = 1;
    ctx->nchunk = (int)std::min<long long>(std::min<long long>(std::max<long long>(1, (2048 + tblocks - 1) / tblocks),
                                                               ctx->ntiles), kMaxChunks);
    if ((rc = dev_alloc(ctx, &ctx->d_partial, (size_t)kMaxChunks * 9 * T))) return rc;
    if ((rc = dev_alloc(ctx, &ctx->d_info_tmp, ndrops))) return rc;

    // --- target geometry (own grids) and far-source geometry
    return build_geometry(ctx);
}

int ehd_update_shape(ehd_ctx* ctx, const double* xcoef_d)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!xcoef_d || ((uintptr_t)xcoef_d) % 8) EHD_FAIL(ctx, EHD_E_ARG, "xcoef_d must be non-NULL and 8-byte aligned");
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->drop_graph();
    if (xcoef_d != ctx->d_x)
        EHD_HIP(ctx, hipMemcpyAsync(ctx->d_x, xcoef_d, sizeof(double) * 3 * ctx->ncoef_total, hipMemcpyDeviceToDevice,
                                    ctx->stream));
    int rc = read_centres(ctx);
    if (rc) return rc;
    std::vector<double> cen(4 * ctx->nd, 0.0);             // radii: build_geometry
    for (int d = 0; d < ctx->nd; ++d)
        for (int c = 0; c < 3; ++c) cen[4 * d + c] = ctx->info[d].c[c];
    EHD_HIP(ctx, hipMemcpyAsync(ctx->d_centre, cen.data(), sizeof(double) * cen.size(), hipMemcpyHostToDevice,
                                ctx->stream));
    EHD_HIP(ctx, hipMemcpyAsync(ctx->d_info, ctx->info.data(), sizeof(DropInfo) * ctx->info.size(),
                                hipMemcpyHostToDevice, ctx->stream));
    if ((rc = build_geometry(ctx))) return rc;
    return near_build(ctx);
}

int ehd_set_near(ehd_ctx* ctx, double delta, double s_check, int m, int q_check)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!std::isfinite(delta) || delta < 0.0) EHD_FAIL(ctx, EHD_E_ARG, "delta must be >= 0");
    if (delta > 0.0) {
        if (m < 2 || m > kNearMaxM) EHD_FAIL(ctx, EHD_E_ARG, "m must be in [2, %d]", kNearMaxM);
        if (!(s_check > 0.0) || !std::isfinite(s_check) || delta > s_check * (1.0 + 0.5 * (m - 1)))
            EHD_FAIL(ctx, EHD_E_ARG, "need s_check > 0 and delta <= s_check (1 + (m-1)/2): the check points "
                     "must reach past every corrected target");
        for (int d = 0; d < ctx->nd; ++d)
            if (q_check < ctx->p[d] || q_check > EHD_MAX_Q_CHECK)
                EHD_FAIL(ctx, EHD_E_ARG, "q_check must be in [p, %d] for every drop", EHD_MAX_Q_CHECK);
    }
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->drop_graph();
    ctx->near.on = delta > 0.0;
    ctx->near.delta = delta;
    ctx->near.sc = s_check;
    ctx->near.m = m;
    ctx->near.qc = q_check;
    return near_build(ctx);
}

int ehd_near_pairs(const ehd_ctx* ctx, long long* npairs)
{
    if (!ctx || !npairs) return EHD_E_ARG;
    *npairs = ctx->near.npairs;
    return ctx->nd ? EHD_OK : EHD_E_STATE;
}

int ehd_num_targets(const ehd_ctx* ctx, long long* ntargets)
{
    if (!ctx || !ntargets) return EHD_E_ARG;
    *ntargets = ctx->T;
    return ctx->nd ? EHD_OK : EHD_E_STATE;
}

int ehd_num_coefs(const ehd_ctx* ctx, long long* ncoef)
{
    if (!ctx || !ncoef) return EHD_E_ARG;
    if (!ctx->nd) return EHD_E_STATE;
    long long n = 0;
    for (int d = 0; d < ctx->nd; ++d) n += (long long)(ctx->info[d].p + 1) * (ctx->info[d].p + 2);
    *ncoef = n;
    return EHD_OK;
}

// Far-field launch with the context's tile shape (targets per thread, source
// chunks) on the context's launch stream.
// Number of far-field work items (target block, chunk) of a tile shape.
static long long far_items(const ehd_ctx* ctx, int tpt, int nchunk)
{
    return (ctx->T + (long long)kThreads * tpt - 1) / ((long long)kThreads * tpt) * nchunk;
}

// Far-field items [vb0, vb1) (vb1 < 0: all), on `blocks` looping blocks
// (0: one block per item).
static int launch_far(ehd_ctx* ctx, int far_prec, unsigned kinds, int tpt, int nchunk, long long vb0 = 0,
                      long long vb1 = -1, long long blocks = 0)
{
    const long long T = ctx->T, S = ctx->Spad;
    const long long tblocks = (T + (long long)kThreads * tpt - 1) / ((long long)kThreads * tpt);
    const long long nvb = tblocks * nchunk;
    if (vb1 < 0) vb1 = nvb;
    if (nvb > INT_MAX) EHD_FAIL(ctx, EHD_E_SHAPE, "too many far-field work items (%lld)", nvb);
    if (vb1 <= vb0) return EHD_OK;
    const int tpc = (ctx->ntiles + nchunk - 1) / nchunk;
    const dim3 grid((unsigned)(blocks > 0 ? std::min(blocks, vb1 - vb0) : vb1 - vb0));
    if (far_prec == EHD_FAR_FP64) {
        const Far64Launch fn = (tpt == 2 ? far64_table<2>() : far64_table<1>())[kinds & EHD_ALL_KINDS];
        fn(grid, ctx->ls, ctx->d_tx, ctx->d_tn, ctx->d_tdrop, T, ctx->d_src64, S, ctx->d_tile_info, ctx->ntiles, tpc,
           ctx->d_partial, (int)tblocks, (int)vb0, (int)vb1);
    } else {
        const Far32Launch fn = (tpt == 2 ? far32_table<2>() : far32_table<1>())[kinds & EHD_ALL_KINDS];
        fn(grid, ctx->ls, ctx->d_tx, ctx->d_tn, ctx->d_tdrop, T, ctx->d_src32, S, ctx->d_tile_info, ctx->d_centre,
           ctx->ntiles, tpc, ctx->d_partial, (int)tblocks, (int)vb0, (int)vb1);
    }
    EHD_HIP(ctx, hipGetLastError());
    return EHD_OK;
}

// Algorithmic FP64 work of one drop's singular self-interaction: rotation of
// 7 fields, Legendre sums of 10 fields, longitude sums of 13 quantities and
// about 75 flops of kernel per rotated node.
static double self_work(const DropInfo& D)
{
    const double T = (double)(D.p + 1) * D.nlon_p, q1 = D.qs + 1.0;
    double rot = 0.0;
    for (int n = 0; n <= D.p; ++n) rot += (n + 1.0) * (2.0 * n + 1.0);
    rot *= 4.0 * 7.0 * T;
    const double leg = 4.0 * q1 * (double)ncoef(D.p) * 10.0 * T;
    const double dft = 2.0 * D.nlon_s * (2.0 * D.p + 1.0) * q1 * 13.0 * T;
    const double ker = 75.0 * T * q1 * D.nlon_s;
    return rot + leg + dft + ker;
}

// Registers per lane (rounded up to the allocation granule of 8) and static
// LDS bytes of a kernel as built; a kernel the runtime cannot describe fits
// beside nothing.
static ehd_ctx::KernRes kernel_res(ehd_ctx* ctx, const void* fn)
{
    auto it = ctx->kres.find(fn);
    if (it != ctx->kres.end()) return it->second;
    ehd_ctx::KernRes r{512, 1 << 30};
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, fn) == hipSuccess) r = {(a.numRegs + 7) / 8 * 8, (int)a.sharedSizeBytes};
    else (void)hipGetLastError();
    ctx->kres.emplace(fn, r);
    return r;
}

// Overlap mode: the degree classes below p = 48 whose blocks leave room on a
// compute unit for one looping FP32 far-field block: each SIMD holds the
// block's two waves of the self-interaction and one far-field wave in its
// 512 registers per lane, and the LDS of both blocks fits the CU's.  A
// class without that room would have its CUs taken by the far-field blocks
// and slow down several times over, so it runs before the fork.  Every
// kernel the evaluation launches for the class must fit.
static unsigned classes_beside_far(ehd_ctx* ctx, int far_prec, unsigned kinds, bool needF, bool needU, bool needLap)
{
    if (far_prec == EHD_FAR_FP64) return 0u;
    struct V { bool hf, hu, hs; };
    V v[2];
    int nv = 0;
    if (needU && (needF || needLap)) { v[nv++] = {needF, false, needLap}; v[nv++] = {false, true, false}; }
    else if (needU) v[nv++] = {false, true, false};
    else v[nv++] = {needF, false, needLap};
    const ehd_ctx::KernRes fr = kernel_res(ctx, far32_kernel(ctx->far_tpt, kinds));
    constexpr int self_waves = SelfClass<16>::NT / 256, far_waves = kThreads / 256;   // per SIMD
    unsigned m = 0;
    for (int c = 0; c < 3; ++c) {
        if (ctx->cls_drops[c].empty()) continue;
        bool fits = true;
        for (int i = 0; i < nv; ++i) {
            const ehd_ctx::KernRes sr =
                kernel_res(ctx, self_kernel_of_class(c, v[i].hf, v[i].hu, v[i].hs, ctx->self_pf[c]));
            const int nf = 3 + (v[i].hf ? 3 : 0) + (v[i].hu ? 3 : 0) + (v[i].hs ? 1 : 0);
            const size_t lds = self_lds_bytes(ctx, ctx->cls_drops[c], nf) + (size_t)sr.lds + (size_t)fr.lds;
            fits = fits && self_waves * sr.vgpr + far_waves * fr.vgpr <= 512 && lds <= (size_t)ctx->max_lds;
        }
        if (fits) m |= 1u << c;
    }
    return m;
}

// Overlap mode: share of the far field's work items forked beside the
// degree classes in `beside`, the expected time of those classes over that
// of the far field (each its algorithmic work over the fraction of peak it
// reaches alone: 0.25, 0.48, 0.65 for the classes, 0.96 for the FP32 far
// field at 53 flops per interaction), at most one half.  The FP64 far field
// needs the same FP64 units as the self-interaction, which slows down by
// about as much as the far work done beside it (256 drops lost 3-8% at
// shares 0.13 and 0.35): share 0.
static double overlap_share(const ehd_ctx* ctx, int far_prec, unsigned beside)
{
    if (far_prec == EHD_FAR_FP64 || !beside) return 0.0;
    static const double eff[3] = {0.25, 0.48, 0.65};
    double small = 0.0, far = 0.0;
    long long S = 0;
    for (int d = 0; d < ctx->nd; ++d) S += ctx->info[d].ns;
    for (int c = 0; c < 3; ++c)
        if (beside & (1u << c))
            for (int d : ctx->cls_drops[c]) small += self_work(ctx->info[d]) / eff[c];
    for (int d = 0; d < ctx->nd; ++d) {
        const DropInfo& D = ctx->info[d];
        far += (double)(D.p + 1) * D.nlon_p * (double)(S - D.ns);
    }
    far *= 53.0 / 0.96;
    return far > 0.0 ? std::min(0.5, small / far) : 0.0;
}

// Overlap mode.  A far field of at most two work items per compute unit
// forks whole, before the self-interaction: its blocks take a few CUs and
// the self-interaction the rest.  A larger one would hold every CU until it
// drains, so it forks as one looping block per CU over a first share of its
// items (overlap_share) beside the degree classes that leave room for such
// a block (classes_beside_far); the other classes run before the fork, and
// the rest of the far field follows on the main stream as an ordinary
// launch.  Every item is summed as in the serial order.  split = the number
// of items forked (0: serial order).
struct OverlapPlan {
    long long nvb = 0, split = 0;
    unsigned beside = 0;
    bool whole = false;
};
static OverlapPlan overlap_plan(ehd_ctx* ctx, int far_prec, unsigned kinds, bool needF, bool needU, bool needLap)
{
    OverlapPlan pl;
    pl.nvb = far_items(ctx, ctx->far_tpt, ctx->nchunk);
    if (!ctx->overlap || ctx->nd < 2) return pl;   // one drop: no far interactions, nothing to overlap
    pl.whole = pl.nvb <= 2LL * ctx->ncu;
    if (pl.whole) {
        for (int c = 0; c < 4; ++c)
            if (!ctx->cls_drops[c].empty()) pl.beside |= 1u << c;
        pl.split = pl.nvb;
    } else {
        pl.beside = classes_beside_far(ctx, far_prec, kinds, needF, needU, needLap);
        pl.split = (long long)std::ceil(overlap_share(ctx, far_prec, pl.beside) * (double)pl.nvb);
        if (pl.split == 0) pl.beside = 0;
    }
    return pl;
}

// The launch sequence of one evaluation, on ctx->ls.
static int enqueue_evaluation(ehd_ctx* ctx, const double* fcoef_d, const double* ucoef_d,
                              const double* sigcoef_d, unsigned kinds, int far_prec, double* self_out_d,
                              double* far_out_d)
{
    const bool needS = kinds & EHD_STOKES_SL, needD = kinds & EHD_STOKES_DL;
    const bool needLap = kinds & (EHD_LAP_SL | EHD_LAP_DL | EHD_LAP_DLADJ);
    const bool needF = needS || (needD && !ucoef_d);
    const bool needU = needD && ucoef_d;
    RowMap rows{};
    for (int c = 0; c < 9; ++c) {
        const unsigned bit = c < 3 ? EHD_STOKES_SL : c < 6 ? EHD_STOKES_DL : c == 6 ? EHD_LAP_SL
                             : c == 7 ? EHD_LAP_DL : EHD_LAP_DLADJ;
        if (kinds & bit) rows.comp[rows.n++] = c;
    }

    const long long T = ctx->T, S = ctx->Spad, vs = ctx->syn_stride;
    ctx->mark(0);
    // 1. densities on the far grids -> weighted source records
    double* synf = needF ? ctx->d_syn : nullptr;
    double* synu = needU ? ctx->d_syn + 3 * vs : nullptr;
    double* syns = needLap ? ctx->d_syn + 6 * vs : nullptr;
    if (needF)
        hipLaunchKernelGGL((k_synth<3, false>), dim3(ctx->nrows_f), dim3(kThreads), 0, ctx->ls, ctx->d_info,
                           ctx->d_legs, 1, ctx->d_rows_f, fcoef_d, synf, vs);
    if (needU)
        hipLaunchKernelGGL((k_synth<3, false>), dim3(ctx->nrows_f), dim3(kThreads), 0, ctx->ls, ctx->d_info,
                           ctx->d_legs, 1, ctx->d_rows_f, ucoef_d, synu, vs);
    if (needLap)
        hipLaunchKernelGGL((k_synth<1, false>), dim3(ctx->nrows_f), dim3(kThreads), 0, ctx->ls, ctx->d_info,
                           ctx->d_legs, 1, ctx->d_rows_f, sigcoef_d, syns, vs);
    hipLaunchKernelGGL(k_src_dens, dim3((S + 255) / 256), dim3(256), 0, ctx->ls, synf, synu, syns, vs, S,
                       ctx->d_src64, ctx->d_src32);
    EHD_HIP(ctx, hipGetLastError());

    ctx->mark(1);
    // 2. singular self-interaction.  The kernel holds at most 8 fields (its
    //    Legendre MFMA has 16 columns: field x re/im), so a separate u goes
    //    through its own pass (x, u) for D while the first pass covers the
    //    other kinds.
    // the nearly singular correction of K* needs the single layer's on-surface values
    const unsigned kself = (ctx->near.npairs && (kinds & EHD_LAP_DLADJ)) ? (kinds | EHD_LAP_SL) : kinds;
    auto self_classes = [&](unsigned cm) {
        int rc = EHD_OK;
        if (needU && (needF || needLap)) {
            const unsigned k1 = kself & ~(unsigned)EHD_STOKES_DL;
            if (needF && needLap) rc = launch_self<true, false, true>(ctx, fcoef_d, nullptr, sigcoef_d, k1, cm);
            else if (needF) rc = launch_self<true, false, false>(ctx, fcoef_d, nullptr, sigcoef_d, k1, cm);
            else rc = launch_self<false, false, true>(ctx, fcoef_d, nullptr, sigcoef_d, k1, cm);
            if (rc == EHD_OK)
                rc = launch_self<false, true, false>(ctx, fcoef_d, ucoef_d, sigcoef_d, EHD_STOKES_DL, cm);
        } else if (needU) {
            rc = launch_self<false, true, false>(ctx, fcoef_d, ucoef_d, sigcoef_d, kself, cm);
        } else if (needF && needLap) {
            rc = launch_self<true, false, true>(ctx, fcoef_d, ucoef_d, sigcoef_d, kself, cm);
        } else if (needF) {
            rc = launch_self<true, false, false>(ctx, fcoef_d, ucoef_d, sigcoef_d, kself, cm);
        } else {
            rc = launch_self<false, false, true>(ctx, fcoef_d, ucoef_d, sigcoef_d, kself, cm);
        }
        return rc;
    };
    const OverlapPlan pl = overlap_plan(ctx, far_prec, kinds, needF, needU, needLap);
    const long long nvb = pl.nvb, split = pl.split;
    const bool whole = pl.whole;
    const unsigned beside = whole ? 0xFu : pl.beside;
    int rc;
    if (split == 0) {
        if ((rc = self_classes(0xFu))) return rc;
        ctx->mark(2);
        // 3. far field
        if ((rc = launch_far(ctx, far_prec, kinds, ctx->far_tpt, ctx->nchunk))) return rc;
    } else {
        if (!whole && (rc = self_classes(0xFu & ~beside))) return rc;
        EHD_HIP(ctx, hipEventRecord(ctx->ev_fork, ctx->ls));
        EHD_HIP(ctx, hipStreamWaitEvent(ctx->far_stream, ctx->ev_fork, 0));
        hipStream_t main = ctx->ls;
        ctx->ls = ctx->far_stream;
        rc = launch_far(ctx, far_prec, kinds, ctx->far_tpt, ctx->nchunk, 0, split, whole ? 0 : ctx->ncu);
        ctx->ls = main;
        if (rc) return rc;
        EHD_HIP(ctx, hipEventRecord(ctx->ev_join, ctx->far_stream));
        if ((rc = self_classes(beside))) return rc;
        ctx->mark(2);
        // 3. far field: the rest, then the forked part
        if ((rc = launch_far(ctx, far_prec, kinds, ctx->far_tpt, ctx->nchunk, split, nvb))) return rc;
        EHD_HIP(ctx, hipStreamWaitEvent(ctx->ls, ctx->ev_join, 0));
    }

    ctx->mark(3);
    // 4. outputs
    hipLaunchKernelGGL(k_combine, dim3((T + 255) / 256), dim3(256), 0, ctx->ls, ctx->d_raw, ctx->d_partial,
                       ctx->nchunk, T, rows, self_out_d, far_out_d);
    EHD_HIP(ctx, hipGetLastError());
    // 5. nearly singular targets: replace the affected drops' far sums
    if (ctx->near.npairs) {
        const double* fc = (needF || (needD && !ucoef_d)) ? fcoef_d : nullptr;
        const double* uc = needU ? ucoef_d : nullptr;
        if ((rc = near_enqueue(ctx, fc, uc, needLap ? sigcoef_d : nullptr, rows, far_out_d ? far_out_d : self_out_d)))
            return rc;
    }
    ctx->mark(4);
    return EHD_OK;
}

int ehd_layer_potentials(ehd_ctx* ctx, const double* fcoef_d, const double* ucoef_d,
                         const double* sigcoef_d, unsigned kinds, int far_prec, double* self_out_d,
                         double* far_out_d)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (kinds == 0 || (kinds & ~(unsigned)EHD_ALL_KINDS)) EHD_FAIL(ctx, EHD_E_ARG, "invalid kinds mask 0x%x", kinds);
    if (far_prec != EHD_FAR_FP64 && far_prec != EHD_FAR_FP32C) EHD_FAIL(ctx, EHD_E_ARG, "invalid far_prec %d", far_prec);
    if (!self_out_d) EHD_FAIL(ctx, EHD_E_ARG, "self_out_d is NULL");
    const bool needS = kinds & EHD_STOKES_SL, needD = kinds & EHD_STOKES_DL;
    const bool needLap = kinds & (EHD_LAP_SL | EHD_LAP_DL | EHD_LAP_DLADJ);
    const bool needF = needS || (needD && !ucoef_d);
    if (needF && !fcoef_d) EHD_FAIL(ctx, EHD_E_ARG, "fcoef_d is needed for the requested kinds");
    if (needLap && !sigcoef_d) EHD_FAIL(ctx, EHD_E_ARG, "sigcoef_d is needed for the Laplace kinds");
    for (const void* q : {(const void*)fcoef_d, (const void*)ucoef_d, (const void*)sigcoef_d,
                          (const void*)self_out_d, (const void*)far_out_d})
        if (((uintptr_t)q) % 8) EHD_FAIL(ctx, EHD_E_ARG, "device pointers must be 8-byte aligned");
    EHD_HIP(ctx, hipSetDevice(ctx->device));

    int rc;
    if (!ctx->graph_on) {
        ctx->ls = ctx->stream;
        rc = enqueue_evaluation(ctx, fcoef_d, ucoef_d, sigcoef_d, kinds, far_prec, self_out_d, far_out_d);
    } else {
        const ehd_ctx::GraphKey key{fcoef_d, ucoef_d, sigcoef_d, self_out_d, far_out_d, kinds, far_prec,
                                    ctx->far_tpt, ctx->nchunk};
        if (!ctx->gexec || !(key == ctx->gkey)) {
            ctx->drop_graph();
            // record the sequence on the private stream, then instantiate
            ctx->ls = ctx->cap_stream;
            ctx->capturing = true;
            hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) {
                ctx->capturing = false;
                EHD_FAIL(ctx, EHD_E_HIP, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
            }
            rc = enqueue_evaluation(ctx, fcoef_d, ucoef_d, sigcoef_d, kinds, far_prec, self_out_d, far_out_d);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(ctx->cap_stream, &g);
            ctx->capturing = false;
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) EHD_FAIL(ctx, EHD_E_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                ctx->gexec = nullptr;
                EHD_FAIL(ctx, EHD_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
            }
            ctx->gkey = key;
        }
        ctx->mark(0);
        EHD_HIP(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
        for (int k = 1; k <= ehd_ctx::kStages; ++k) ctx->mark(k);
        rc = EHD_OK;
    }
    if (rc) return rc;
    if (ctx->nslots) {
        const long long slot = ctx->ncalls % ctx->nslots;
        ctx->slot_used[slot] = 1;
    }
    ++ctx->ncalls;
    return EHD_OK;
}

int ehd_set_graph(ehd_ctx* ctx, int enable)
{
    if (!ctx) return EHD_E_ARG;
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    if (ctx->stream) EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->drop_graph();
    if (enable && !ctx->cap_stream)
        EHD_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    ctx->graph_on = enable != 0;
    return EHD_OK;
}

int ehd_set_overlap(ehd_ctx* ctx, int enable)
{
    if (!ctx) return EHD_E_ARG;
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    if (ctx->stream) EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->drop_graph();
    if (enable && !ctx->far_stream) {
        EHD_HIP(ctx, hipStreamCreateWithFlags(&ctx->far_stream, hipStreamNonBlocking));
        EHD_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
        EHD_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    }
    ctx->overlap = enable != 0;
    return EHD_OK;
}

int ehd_overlap_plan(ehd_ctx* ctx, unsigned kinds, int far_prec, int with_u, unsigned* beside, long long* forked)
{
    if (!ctx || !beside || !forked) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "no drops set");
    if (far_prec != EHD_FAR_FP64 && far_prec != EHD_FAR_FP32C) EHD_FAIL(ctx, EHD_E_ARG, "unknown far precision");
    if (!(kinds & EHD_ALL_KINDS) || (kinds & ~(unsigned)EHD_ALL_KINDS)) EHD_FAIL(ctx, EHD_E_ARG, "bad kinds mask");
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    const bool needS = kinds & EHD_STOKES_SL, needD = kinds & EHD_STOKES_DL;
    const bool needLap = kinds & (EHD_LAP_SL | EHD_LAP_DL | EHD_LAP_DLADJ);
    const OverlapPlan pl = overlap_plan(ctx, far_prec, kinds, needS || (needD && !with_u), needD && with_u, needLap);
    *beside = pl.split ? pl.beside : 0u;
    *forked = pl.split;
    return EHD_OK;
}

int ehd_set_far_config(ehd_ctx* ctx, int targets_per_thread, int nchunk)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if ((targets_per_thread != 1 && targets_per_thread != 2) || nchunk < 1 || nchunk > kMaxChunks ||
        nchunk > ctx->ntiles)
        EHD_FAIL(ctx, EHD_E_ARG, "targets_per_thread must be 1 or 2 and nchunk in [1, %d] (and <= %d tiles)",
                 kMaxChunks, ctx->ntiles);
    ctx->far_tpt = targets_per_thread;
    ctx->nchunk = nchunk;
    return EHD_OK;
}

int ehd_get_far_config(const ehd_ctx* ctx, int* targets_per_thread, int* nchunk)
{
    if (!ctx || !targets_per_thread || !nchunk) return EHD_E_ARG;
    *targets_per_thread = ctx->far_tpt;
    *nchunk = ctx->nchunk;
    return ctx->nd ? EHD_OK : EHD_E_STATE;
}

int ehd_time_far(ehd_ctx* ctx, int far_prec, unsigned kinds, int targets_per_thread, int nchunk, int reps,
                 double* ms)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!ms || reps < 1 || reps > 1000 || (far_prec != EHD_FAR_FP64 && far_prec != EHD_FAR_FP32C))
        EHD_FAIL(ctx, EHD_E_ARG, "invalid arguments");
    if (kinds == 0 || (kinds & ~(unsigned)EHD_ALL_KINDS)) EHD_FAIL(ctx, EHD_E_ARG, "invalid kinds mask 0x%x", kinds);
    if ((targets_per_thread != 1 && targets_per_thread != 2) || nchunk < 1 || nchunk > kMaxChunks ||
        nchunk > ctx->ntiles)
        EHD_FAIL(ctx, EHD_E_ARG, "invalid tile shape");
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    hipEvent_t e0, e1;
    EHD_HIP(ctx, hipEventCreate(&e0));
    EHD_HIP(ctx, hipEventCreate(&e1));
    ctx->ls = ctx->stream;
    int rc = launch_far(ctx, far_prec, kinds, targets_per_thread, nchunk);  // warm-up
    if (!rc) {
        (void)hipEventRecord(e0, ctx->stream);
        for (int r = 0; r < reps && !rc; ++r) rc = launch_far(ctx, far_prec, kinds, targets_per_thread, nchunk);
        (void)hipEventRecord(e1, ctx->stream);
        (void)hipEventSynchronize(e1);
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = t / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// Self-interaction prefetch batches built per degree class: the default
// first, then the two alternatives (field set x, f, sigma only).
static void self_pf_candidates(int cls, int* pf)
{
    switch (cls) {
    case 0: pf[0] = SelfClass<16>::PF; pf[1] = SelfClass<16>::PF_ALT0; pf[2] = SelfClass<16>::PF_ALT1; break;
    case 1: pf[0] = SelfClass<24>::PF; pf[1] = SelfClass<24>::PF_ALT0; pf[2] = SelfClass<24>::PF_ALT1; break;
    case 2: pf[0] = SelfClass<32>::PF; pf[1] = SelfClass<32>::PF_ALT0; pf[2] = SelfClass<32>::PF_ALT1; break;
    default: pf[0] = SelfClass<48>::PF; pf[1] = SelfClass<48>::PF_ALT0; pf[2] = SelfClass<48>::PF_ALT1; break;
    }
}

int ehd_self_config_candidates(int cls, int* pf, int* n)
{
    if (cls < 0 || cls > 3 || !pf || !n) return EHD_E_ARG;
    self_pf_candidates(cls, pf);
    *n = 3;
    return EHD_OK;
}

int ehd_set_self_config(ehd_ctx* ctx, int cls, int pf)
{
    if (!ctx) return EHD_E_ARG;
    if (cls < 0 || cls > 3) EHD_FAIL(ctx, EHD_E_ARG, "degree class must be 0..3");
    int c[3];
    self_pf_candidates(cls, c);
    if (pf != 0 && pf != c[0] && pf != c[1] && pf != c[2])
        EHD_FAIL(ctx, EHD_E_ARG, "prefetch batch %d is not built for class %d (0, %d, %d or %d)", pf, cls, c[0], c[1],
                 c[2]);
    const int eff = pf == c[0] ? 0 : pf;
    if (ctx->self_pf[cls] != eff) {
        if (ctx->stream) EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
        ctx->drop_graph();
        ctx->self_pf[cls] = eff;
    }
    return EHD_OK;
}

int ehd_get_self_config(const ehd_ctx* ctx, int cls, int* pf)
{
    if (!ctx || cls < 0 || cls > 3 || !pf) return EHD_E_ARG;
    int c[3];
    self_pf_candidates(cls, c);
    *pf = ctx->self_pf[cls] ? ctx->self_pf[cls] : c[0];
    return EHD_OK;
}

int ehd_time_self(ehd_ctx* ctx, int cls, int pf, const double* fcoef_d, const double* sigcoef_d, int reps, double* ms)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!ms || !fcoef_d || !sigcoef_d || reps < 1 || reps > 1000) EHD_FAIL(ctx, EHD_E_ARG, "invalid arguments");
    if (cls < 0 || cls > 3) EHD_FAIL(ctx, EHD_E_ARG, "degree class must be 0..3");
    const int keep = ctx->self_pf[cls];
    int rc = ehd_set_self_config(ctx, cls, pf);
    if (rc) return rc;
    *ms = 0.0;
    if (ctx->cls_off[cls + 1] == ctx->cls_off[cls]) return ehd_set_self_config(ctx, cls, keep);
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    hipEvent_t e0, e1;
    EHD_HIP(ctx, hipEventCreate(&e0));
    EHD_HIP(ctx, hipEventCreate(&e1));
    ctx->ls = ctx->stream;
    const unsigned kinds = EHD_STOKES_SL | EHD_STOKES_DL | EHD_LAP_SL | EHD_LAP_DL;
    const unsigned cm = 1u << cls;
    rc = launch_self<true, false, true>(ctx, fcoef_d, nullptr, sigcoef_d, kinds, cm);   // warm-up
    if (!rc) {
        (void)hipEventRecord(e0, ctx->stream);
        for (int r = 0; r < reps && !rc; ++r) rc = launch_self<true, false, true>(ctx, fcoef_d, nullptr, sigcoef_d, kinds, cm);
        (void)hipEventRecord(e1, ctx->stream);
        (void)hipEventSynchronize(e1);
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = t / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int rc2 = ehd_set_self_config(ctx, cls, keep == 0 ? 0 : keep);
    return rc ? rc : rc2;
}

int ehd_surface(ehd_ctx* ctx, int ng, const double* gcoef_d, double* H_d, double* grad_d, double* lap_d)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (ng < 0 || ng > 3) EHD_FAIL(ctx, EHD_E_ARG, "ng must be 0, 1, 2 or 3");
    if (!H_d || (ng > 0 && (!gcoef_d || !grad_d))) EHD_FAIL(ctx, EHD_E_ARG, "NULL pointer");
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    const dim3 grid(ctx->nrows_p), block(kThreads);
    if (ng == 0)
        hipLaunchKernelGGL(k_surface<0>, grid, block, 0, ctx->stream, ctx->d_info, ctx->d_legs, ctx->d_rows_p, ctx->d_x,
                           gcoef_d, ctx->T, H_d, grad_d, lap_d);
    else if (ng == 1)
        hipLaunchKernelGGL(k_surface<1>, grid, block, 0, ctx->stream, ctx->d_info, ctx->d_legs, ctx->d_rows_p, ctx->d_x,
                           gcoef_d, ctx->T, H_d, grad_d, lap_d);
    else if (ng == 2)
        hipLaunchKernelGGL(k_surface<2>, grid, block, 0, ctx->stream, ctx->d_info, ctx->d_legs, ctx->d_rows_p, ctx->d_x,
                           gcoef_d, ctx->T, H_d, grad_d, lap_d);
    else
        hipLaunchKernelGGL(k_surface<3>, grid, block, 0, ctx->stream, ctx->d_info, ctx->d_legs, ctx->d_rows_p, ctx->d_x,
                           gcoef_d, ctx->T, H_d, grad_d, lap_d);
    EHD_HIP(ctx, hipGetLastError());
    return EHD_OK;
}

int ehd_area_weights(ehd_ctx* ctx, double* w_d)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!w_d) EHD_FAIL(ctx, EHD_E_ARG, "w_d is NULL");
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    const long long vs = ctx->syn_stride;
    hipLaunchKernelGGL((k_synth<3, true>), dim3(ctx->nrows_p), dim3(kThreads), 0, ctx->stream,
                       ctx->d_info, ctx->d_legs, 0, ctx->d_rows_p, ctx->d_x, ctx->d_syn, vs);
    hipLaunchKernelGGL(k_area_weights, dim3((ctx->T + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_info,
                       ctx->d_legs, ctx->d_tdrop, ctx->d_syn, vs, ctx->T, w_d);
    EHD_HIP(ctx, hipGetLastError());
    return EHD_OK;
}

int ehd_synthesize(ehd_ctx* ctx, int nfields, const double* coef_d, double* grid_d)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (nfields < 1 || !coef_d || !grid_d) EHD_FAIL(ctx, EHD_E_ARG, "nfields >= 1 and non-NULL pointers required");
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    // One field at a time through the K = 1 kernel on per-field views: field
    // f of drop d starts at nfields*coff[d] + f*(p+1)(p+2) doubles, so each
    // launch reads a descriptor copy whose offsets point there.  Synchronous
    // (the host descriptor copy is reused per field).
    std::vector<DropInfo> shifted(ctx->info);
    DropInfo* d_sh = ctx->d_info_tmp;
    for (int f = 0; f < nfields; ++f) {
        for (int d = 0; d < ctx->nd; ++d)
            shifted[d].coff = (long long)nfields * ctx->info[d].coff + (long long)f * (ctx->info[d].p + 1) * (ctx->info[d].p + 2);
        EHD_HIP(ctx, hipMemcpyAsync(d_sh, shifted.data(), sizeof(DropInfo) * shifted.size(),
                                    hipMemcpyHostToDevice, ctx->stream));
        hipLaunchKernelGGL((k_synth<1, false>), dim3(ctx->nrows_p), dim3(kThreads), 0, ctx->stream, d_sh,
                           ctx->d_legs, 0, ctx->d_rows_p, coef_d, grid_d + (long long)f * ctx->T, ctx->T);
        EHD_HIP(ctx, hipGetLastError());
        EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return EHD_OK;
}

int ehd_analyze(ehd_ctx* ctx, int nfields, const double* grid_d, double* coef_d)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (nfields < 1 || !coef_d || !grid_d) EHD_FAIL(ctx, EHD_E_ARG, "nfields >= 1 and non-NULL pointers required");
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_analyze, dim3(ctx->n_an_items), dim3(kThreads), 0, ctx->stream, ctx->d_info, ctx->d_legs,
                       ctx->d_an_items, nfields, grid_d, ctx->T, coef_d);
    EHD_HIP(ctx, hipGetLastError());
    return EHD_OK;
}

int ehd_drop_coefs(ehd_ctx* ctx, double* xcoef_d)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!xcoef_d) EHD_FAIL(ctx, EHD_E_ARG, "xcoef_d is NULL");
    long long n = 0;
    for (int d = 0; d < ctx->nd; ++d) n += (long long)(ctx->info[d].p + 1) * (ctx->info[d].p + 2);
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    EHD_HIP(ctx, hipMemcpyAsync(xcoef_d, ctx->d_x, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, ctx->stream));
    return EHD_OK;
}

int ehd_target_geometry(ehd_ctx* ctx, double* x_d, double* n_d)
{
    if (!ctx) return EHD_E_ARG;
    if (!ctx->nd) EHD_FAIL(ctx, EHD_E_STATE, "ehd_set_drops has not been called");
    if (!x_d || !n_d) EHD_FAIL(ctx, EHD_E_ARG, "x_d and n_d must be non-NULL");
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    EHD_HIP(ctx, hipMemcpyAsync(x_d, ctx->d_tx, sizeof(double) * 3 * ctx->T, hipMemcpyDeviceToDevice, ctx->stream));
    EHD_HIP(ctx, hipMemcpyAsync(n_d, ctx->d_tn, sizeof(double) * 3 * ctx->T, hipMemcpyDeviceToDevice, ctx->stream));
    return EHD_OK;
}

int ehd_set_timing(ehd_ctx* ctx, int nslots)
{
    if (!ctx) return EHD_E_ARG;
    if (nslots < 0 || nslots > 100000) EHD_FAIL(ctx, EHD_E_ARG, "nslots must be in [0, 100000]");
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    if (ctx->stream) EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->free_events();
    if (nslots == 0) return EHD_OK;
    ctx->events.resize((size_t)nslots * ehd_ctx::kEv);
    for (auto& e : ctx->events) EHD_HIP(ctx, hipEventCreate(&e));
    ctx->slot_used.assign(nslots, 0);
    ctx->class_used.assign((size_t)nslots * 4, 0);
    ctx->nslots = nslots;
    ctx->ncalls = 0;
    return EHD_OK;
}

int ehd_stage_times(ehd_ctx* ctx, int slot, double* ms)
{
    if (!ctx) return EHD_E_ARG;
    if (!ms || slot < 0 || slot >= ctx->nslots) EHD_FAIL(ctx, EHD_E_ARG, "invalid slot or ms pointer");
    if (!ctx->slot_used[slot]) EHD_FAIL(ctx, EHD_E_STATE, "slot %d holds no recorded call", slot);
    hipEvent_t* ev = &ctx->events[(size_t)slot * ehd_ctx::kEv];
    EHD_HIP(ctx, hipEventSynchronize(ev[ehd_ctx::kStages]));
    for (int k = 0; k < ehd_ctx::kStages; ++k) {
        float t = 0.0f;
        EHD_HIP(ctx, hipEventElapsedTime(&t, ev[k], ev[k + 1]));
        ms[k] = t;
    }
    return EHD_OK;
}

int ehd_self_class_times(ehd_ctx* ctx, int slot, double* ms)
{
    if (!ctx) return EHD_E_ARG;
    if (!ms || slot < 0 || slot >= ctx->nslots) EHD_FAIL(ctx, EHD_E_ARG, "invalid slot or ms pointer");
    if (!ctx->slot_used[slot]) EHD_FAIL(ctx, EHD_E_STATE, "slot %d holds no recorded call", slot);
    hipEvent_t* ev = &ctx->events[(size_t)slot * ehd_ctx::kEv];
    EHD_HIP(ctx, hipEventSynchronize(ev[ehd_ctx::kStages]));
    for (int c = 0; c < 4; ++c) {
        ms[c] = 0.0;
        if (!ctx->class_used[(size_t)slot * 4 + c]) continue;
        float t = 0.0f;
        EHD_HIP(ctx, hipEventElapsedTime(&t, ev[ehd_ctx::kStages + 1 + 2 * c], ev[ehd_ctx::kStages + 2 + 2 * c]));
        ms[c] = t;
    }
    return EHD_OK;
}

int ehd_sync(ehd_ctx* ctx)
{
    if (!ctx) return EHD_E_ARG;
    EHD_HIP(ctx, hipSetDevice(ctx->device));
    if (ctx->stream) EHD_HIP(ctx, hipStreamSynchronize(ctx->stream));
    else EHD_HIP(ctx, hipDeviceSynchronize());
    EHD_HIP(ctx, hipGetLastError());
    return EHD_OK;
}

}  // extern "C"
