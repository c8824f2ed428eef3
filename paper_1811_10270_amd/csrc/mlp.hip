// Multilayer perceptron for the learned GMRES initial guess: nlayers hidden
// layers of nhidden ReLU units and a linear output, FP32, trained with Adam
// on a mean-squared error.  Every step runs in the kernels of this file:
// the GEMMs on FP32 MFMA (v_mfma_f32_16x16x4f32; one wave computes a 32x32
// tile as 2x2 MFMA tiles, operands read from global memory with strides, so
// one kernel covers X W, dZ W^T and X^T dZ), the bias/ReLU epilogue, the ReLU
// mask, the bias-gradient column sums, the loss and its gradient, and Adam.
//
// Parameter layout (host and device): for each layer l (0 .. nlayers), the
// weights W_l [in_l][out_l] row-major, then the bias b_l [out_l].

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "ehdbim.h"

struct ehd_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    int nin = 0, nhid = 0, nlay = 0, nout = 0;
    std::vector<int> din, dout;         // per layer
    std::vector<long long> woff, boff;  // offsets into the parameter vector
    long long nparam = 0;
    float *w = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    long long adam_t = 0;
    int cap = 0;                        // batch capacity of the activations
    std::vector<float*> act;            // act[0] = input copy, act[l+1] = output of layer l
    float *dA = nullptr, *dB = nullptr; // backward scratch [cap][max width]
    float* red = nullptr;               // loss reduction scratch
    std::string err;
};

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kT = 256;

// C[M][N] = sum_k A(i,k) B(k,j) (+ bias[j]) (ReLU if relu), A(i,k) =
// A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj], C row-major.  Block: 4 waves,
// a 64x64 tile; wave: 32x32 (2x2 MFMA tiles of 16x16).  MFMA f32 16x16x4:
// lane holds A[lane%16][lane/16] and B[lane/16][lane%16]; element r of the
// result is row 4 (lane/16) + r, column lane%16.
__global__ __launch_bounds__(kT) void k_gemm(const float* __restrict__ A, long long sai, long long sak,
                                             const float* __restrict__ B, long long sbk, long long sbj,
                                             float* __restrict__ C, const float* __restrict__ bias, int relu,
                                             int M, int N, int K)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i0 = blockIdx.y * 64 + (wv >> 1) * 32, j0 = blockIdx.x * 64 + (wv & 1) * 32;
    f4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f4{0, 0, 0, 0};
    const int r16 = lane & 15, k4 = lane >> 4;
    for (int k = 0; k < K; k += 4) {
        const int kk = k + k4;
        float av[2], bv[2];
        for (int a = 0; a < 2; ++a) {
            const int i = i0 + 16 * a + r16;
            av[a] = (i < M && kk < K) ? A[i * sai + kk * sak] : 0.0f;
        }
        for (int b = 0; b < 2; ++b) {
            const int j = j0 + 16 * b + r16;
            bv[b] = (j < N && kk < K) ? B[kk * sbk + j * sbj] : 0.0f;
        }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int j = j0 + 16 * b + r16;
            if (j >= N) continue;
            const float bb = bias ? bias[j] : 0.0f;
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * a + 4 * k4 + r;
                if (i >= M) continue;
                float v = acc[a][b][r] + bb;
                if (relu) v = v > 0.0f ? v : 0.0f;
                C[(long long)i * N + j] = v;
            }
        }
}

// dz = dh where h > 0, else 0
__global__ void k_relu_mask(const float* __restrict__ h, const float* __restrict__ dh, float* __restrict__ dz,
                            long long n)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dz[t] = h[t] > 0.0f ? dh[t] : 0.0f;
}

// db[j] = sum_i dz[i][j] (fixed order)
__global__ void k_colsum(const float* __restrict__ dz, int M, int N, float* __restrict__ db)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.0f;
    for (int i = 0; i < M; ++i) s += dz[(long long)i * N + j];
    db[j] = s;
}

// dy = 2 (y - t) / n and per-block partial sums of (y - t)^2
__global__ __launch_bounds__(kT) void k_mse(const float* __restrict__ y, const float* __restrict__ t, long long n,
                                            float* __restrict__ dy, float* __restrict__ part)
{
    const long long i = (long long)blockIdx.x * kT + threadIdx.x;
    float e = 0.0f;
    if (i < n) {
        const float d = y[i] - t[i];
        dy[i] = 2.0f * d / (float)n;
        e = d * d;
    }
    __shared__ float sh[kT];
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, long long n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi, b = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    w[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

unsigned nb(long long n) { return (unsigned)((n + kT - 1) / kT); }

int fail(ehd_mlp* mlp, int code, const char* msg)
{
    if (mlp) mlp->err = msg;
    return code;
}

#define MLP_HIP(call)                                                                           \
    do {                                                                                        \
        hipError_t _e = (call);                                                                 \
        if (_e != hipSuccess) {                                                                 \
            char _b[256];                                                                       \
            snprintf(_b, sizeof(_b), "%s failed: %s", #call, hipGetErrorString(_e));            \
            return fail(mlp, EHD_E_HIP, _b);                                                    \
        }                                                                                       \
    } while (0)

int gemm(ehd_mlp* mlp, const float* A, long long sai, long long sak, const float* B, long long sbk, long long sbj,
         float* C, const float* bias, int relu, int M, int N, int K)
{
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    hipLaunchKernelGGL(k_gemm, grid, dim3(kT), 0, mlp->stream, A, sai, sak, B, sbk, sbj, C, bias, relu, M, N, K);
    MLP_HIP(hipGetLastError());
    return EHD_OK;
}

int ensure_capacity(ehd_mlp* mlp, int batch)
{
    if (batch <= mlp->cap) return EHD_OK;
    MLP_HIP(hipStreamSynchronize(mlp->stream));   // the old buffers may still be in use
    for (float* a : mlp->act)
        if (a) (void)hipFree(a);
    if (mlp->dA) (void)hipFree(mlp->dA);
    if (mlp->dB) (void)hipFree(mlp->dB);
    mlp->act.assign(mlp->nlay + 2, nullptr);
    mlp->dA = mlp->dB = nullptr;
    mlp->cap = 0;
    int wmax = std::max(mlp->nin, std::max(mlp->nhid, mlp->nout));
    MLP_HIP(hipMalloc(&mlp->act[0], sizeof(float) * (size_t)batch * mlp->nin));
    for (int l = 0; l <= mlp->nlay; ++l)
        MLP_HIP(hipMalloc(&mlp->act[l + 1], sizeof(float) * (size_t)batch * mlp->dout[l]));
    MLP_HIP(hipMalloc(&mlp->dA, sizeof(float) * (size_t)batch * wmax));
    MLP_HIP(hipMalloc(&mlp->dB, sizeof(float) * (size_t)batch * wmax));
    mlp->cap = batch;
    return EHD_OK;
}

uint64_t splitmix(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int ehd_mlp_create(ehd_mlp** out, int device, void* stream, int nin, int nhidden, int nlayers, int nout,
                   unsigned long long seed)
{
    if (!out || nin < 1 || nhidden < 1 || nlayers < 0 || nout < 1) return EHD_E_ARG;
    ehd_mlp* mlp = new ehd_mlp;
    *out = nullptr;
    mlp->device = device;
    mlp->stream = (hipStream_t)stream;
    mlp->nin = nin;
    mlp->nhid = nhidden;
    mlp->nlay = nlayers;
    mlp->nout = nout;
    for (int l = 0; l <= nlayers; ++l) {
        mlp->din.push_back(l == 0 ? nin : nhidden);
        mlp->dout.push_back(l == nlayers ? nout : nhidden);
        mlp->woff.push_back(mlp->nparam);
        mlp->nparam += (long long)mlp->din[l] * mlp->dout[l];
        mlp->boff.push_back(mlp->nparam);
        mlp->nparam += mlp->dout[l];
    }
    // He-uniform weights from a counter-based generator, zero biases
    std::vector<float> h((size_t)mlp->nparam, 0.0f);
    uint64_t st = seed;
    for (int l = 0; l <= nlayers; ++l) {
        const double a = std::sqrt(6.0 / mlp->din[l]);
        for (long long i = 0; i < (long long)mlp->din[l] * mlp->dout[l]; ++i) {
            const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
            h[(size_t)(mlp->woff[l] + i)] = (float)((2.0 * u - 1.0) * a);
        }
    }
    if (hipSetDevice(device) != hipSuccess || hipMalloc(&mlp->w, sizeof(float) * h.size()) != hipSuccess ||
        hipMalloc(&mlp->g, sizeof(float) * h.size()) != hipSuccess ||
        hipMalloc(&mlp->m1, sizeof(float) * h.size()) != hipSuccess ||
        hipMalloc(&mlp->m2, sizeof(float) * h.size()) != hipSuccess ||
        hipMalloc(&mlp->red, sizeof(float) * 65536) != hipSuccess ||
        hipMemcpy(mlp->w, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(mlp->g, 0, sizeof(float) * h.size()) != hipSuccess ||
        hipMemset(mlp->m1, 0, sizeof(float) * h.size()) != hipSuccess ||
        hipMemset(mlp->m2, 0, sizeof(float) * h.size()) != hipSuccess) {
        ehd_mlp_destroy(mlp);
        return EHD_E_HIP;
    }
    *out = mlp;
    return EHD_OK;
}

void ehd_mlp_destroy(ehd_mlp* mlp)
{
    if (!mlp) return;
    (void)hipSetDevice(mlp->device);
    for (float* p : {mlp->w, mlp->g, mlp->m1, mlp->m2, mlp->dA, mlp->dB, mlp->red})
        if (p) (void)hipFree(p);
    for (float* a : mlp->act)
        if (a) (void)hipFree(a);
    delete mlp;
}

const char* ehd_mlp_last_error(const ehd_mlp* mlp) { return mlp ? mlp->err.c_str() : "no network"; }

int ehd_mlp_num_params(const ehd_mlp* mlp, long long* n)
{
    if (!mlp || !n) return EHD_E_ARG;
    *n = mlp->nparam;
    return EHD_OK;
}

int ehd_mlp_get_params(ehd_mlp* mlp, float* host)
{
    if (!mlp || !host) return EHD_E_ARG;
    MLP_HIP(hipSetDevice(mlp->device));
    MLP_HIP(hipStreamSynchronize(mlp->stream));
    MLP_HIP(hipMemcpy(host, mlp->w, sizeof(float) * mlp->nparam, hipMemcpyDeviceToHost));
    return EHD_OK;
}

int ehd_mlp_set_params(ehd_mlp* mlp, const float* host)
{
    if (!mlp || !host) return EHD_E_ARG;
    MLP_HIP(hipSetDevice(mlp->device));
    MLP_HIP(hipStreamSynchronize(mlp->stream));
    MLP_HIP(hipMemcpy(mlp->w, host, sizeof(float) * mlp->nparam, hipMemcpyHostToDevice));
    return EHD_OK;
}

int ehd_mlp_get_grads(ehd_mlp* mlp, float* host)
{
    if (!mlp || !host) return EHD_E_ARG;
    MLP_HIP(hipSetDevice(mlp->device));
    MLP_HIP(hipStreamSynchronize(mlp->stream));
    MLP_HIP(hipMemcpy(host, mlp->g, sizeof(float) * mlp->nparam, hipMemcpyDeviceToHost));
    return EHD_OK;
}

int ehd_mlp_forward(ehd_mlp* mlp, int batch, const float* x_d, float* y_d)
{
    if (!mlp || batch < 1 || !x_d) return fail(mlp, EHD_E_ARG, "invalid forward arguments");
    MLP_HIP(hipSetDevice(mlp->device));
    int rc = ensure_capacity(mlp, batch);
    if (rc) return rc;
    MLP_HIP(hipMemcpyAsync(mlp->act[0], x_d, sizeof(float) * (size_t)batch * mlp->nin, hipMemcpyDeviceToDevice,
                           mlp->stream));
    for (int l = 0; l <= mlp->nlay; ++l) {
        const int K = mlp->din[l], N = mlp->dout[l];
        if ((rc = gemm(mlp, mlp->act[l], K, 1, mlp->w + mlp->woff[l], N, 1, mlp->act[l + 1], mlp->w + mlp->boff[l],
                       l < mlp->nlay ? 1 : 0, batch, N, K)))
            return rc;
    }
    if (y_d)
        MLP_HIP(hipMemcpyAsync(y_d, mlp->act[mlp->nlay + 1], sizeof(float) * (size_t)batch * mlp->nout,
                               hipMemcpyDeviceToDevice, mlp->stream));
    return EHD_OK;
}

int ehd_mlp_backward(ehd_mlp* mlp, int batch, const float* dy_d)
{
    if (!mlp || batch < 1 || batch > mlp->cap || !dy_d) return fail(mlp, EHD_E_ARG, "backward needs a forward first");
    MLP_HIP(hipSetDevice(mlp->device));
    int rc;
    // dZ of the output layer is dY
    MLP_HIP(hipMemcpyAsync(mlp->dA, dy_d, sizeof(float) * (size_t)batch * mlp->nout, hipMemcpyDeviceToDevice,
                           mlp->stream));
    for (int l = mlp->nlay; l >= 0; --l) {
        const int K = mlp->din[l], N = mlp->dout[l];
        // dW = H_l^T dZ  ([K][N]), db = column sums of dZ
        if ((rc = gemm(mlp, mlp->act[l], 1, K, mlp->dA, N, 1, mlp->g + mlp->woff[l], nullptr, 0, K, N, batch))) return rc;
        hipLaunchKernelGGL(k_colsum, dim3(nb(N)), dim3(kT), 0, mlp->stream, mlp->dA, batch, N, mlp->g + mlp->boff[l]);
        MLP_HIP(hipGetLastError());
        if (l == 0) break;
        // dH_l = dZ W^T ([batch][K]), then the ReLU mask of layer l-1's output
        if ((rc = gemm(mlp, mlp->dA, N, 1, mlp->w + mlp->woff[l], 1, N, mlp->dB, nullptr, 0, batch, K, N))) return rc;
        hipLaunchKernelGGL(k_relu_mask, dim3(nb((long long)batch * K)), dim3(kT), 0, mlp->stream, mlp->act[l],
                           mlp->dB, mlp->dA, (long long)batch * K);
        MLP_HIP(hipGetLastError());
    }
    return EHD_OK;
}

int ehd_mlp_mse(ehd_mlp* mlp, int batch, const float* y_d, const float* t_d, float* dy_d, double* loss)
{
    if (!mlp || batch < 1 || !y_d || !t_d || !dy_d) return fail(mlp, EHD_E_ARG, "invalid loss arguments");
    const long long n = (long long)batch * mlp->nout;
    if (nb(n) > 65536) return fail(mlp, EHD_E_ARG, "batch too large for the loss reduction");
    MLP_HIP(hipSetDevice(mlp->device));
    hipLaunchKernelGGL(k_mse, dim3(nb(n)), dim3(kT), 0, mlp->stream, y_d, t_d, n, dy_d, mlp->red);
    MLP_HIP(hipGetLastError());
    if (loss) {
        std::vector<float> part(nb(n));
        MLP_HIP(hipMemcpyAsync(part.data(), mlp->red, sizeof(float) * part.size(), hipMemcpyDeviceToHost, mlp->stream));
        MLP_HIP(hipStreamSynchronize(mlp->stream));
        double s = 0.0;
        for (float v : part) s += v;
        *loss = s / (double)n;
    }
    return EHD_OK;
}

int ehd_mlp_adam(ehd_mlp* mlp, float lr, float beta1, float beta2, float eps)
{
    if (!mlp || !(lr > 0.0f)) return fail(mlp, EHD_E_ARG, "invalid Adam arguments");
    MLP_HIP(hipSetDevice(mlp->device));
    ++mlp->adam_t;
    const float c1 = 1.0f - std::pow(beta1, (float)mlp->adam_t), c2 = 1.0f - std::pow(beta2, (float)mlp->adam_t);
    hipLaunchKernelGGL(k_adam, dim3(nb(mlp->nparam)), dim3(kT), 0, mlp->stream, mlp->w, mlp->g, mlp->m1, mlp->m2,
                       mlp->nparam, lr, beta1, beta2, eps, c1, c2);
    MLP_HIP(hipGetLastError());
    return EHD_OK;
}

}  // extern "C"
