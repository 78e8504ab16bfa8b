// Degree picker: a small MLP (66 -> 128 -> 128 -> 128 -> 2, ReLU, FP32) that
// maps Chebyshev (KPM) moments of the scaled matrix and the scaled target
// window to a filter degree and a first filter window.  Forward, backward
// and the Adam update are hand-written kernels; every reduction runs in a
// fixed order (bitwise reproducible).
//
// Parameter layout (one flat FP32 array, FD_MLP_NPARAMS entries): for each
// layer l = 1..4 the weights W_l (n_out x n_in, row-major) then the bias b_l.
#include <cmath>

#include "fd_internal.h"

namespace fd {
namespace {

constexpr int NL = 4;
constexpr int DIMS[NL + 1] = {FD_MLP_IN, FD_MLP_HIDDEN, FD_MLP_HIDDEN, FD_MLP_HIDDEN, FD_MLP_OUT};

int64_t w_off(int l) {  // offset of W_{l+1}, l = 0..3
    int64_t o = 0;
    for (int k = 0; k < l; k++) o += (int64_t)DIMS[k + 1] * DIMS[k] + DIMS[k + 1];
    return o;
}

// Y[i][o] = act(sum_k X[i][k] W[o][k] + b[o]); Z keeps the pre-activation
__global__ void k_dense_fwd(int B, int nin, int nout, const float *__restrict__ X, const float *__restrict__ W,
                            const float *__restrict__ b, float *__restrict__ Z, float *__restrict__ Y, int relu) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * nout) return;
    const int i = e / nout, o = e % nout;
    float s = b[o];
    for (int k = 0; k < nin; k++) s += X[i * nin + k] * W[o * nin + k];
    if (Z) Z[e] = s;
    Y[e] = relu ? fmaxf(s, 0.0f) : s;
}

// dW[o][k] = sum_i dY[i][o] X[i][k];  db[o] = sum_i dY[i][o]
__global__ void k_dense_wgrad(int B, int nin, int nout, const float *__restrict__ X, const float *__restrict__ dY,
                              float *__restrict__ dW, float *__restrict__ db) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nout * (nin + 1)) return;
    const int o = e / (nin + 1), k = e % (nin + 1);
    float s = 0.0f;
    if (k < nin) {
        for (int i = 0; i < B; i++) s += dY[i * nout + o] * X[i * nin + k];
        dW[o * nin + k] = s;
    } else {
        for (int i = 0; i < B; i++) s += dY[i * nout + o];
        db[o] = s;
    }
}

// dX[i][k] = (sum_o dY[i][o] W[o][k]) * relu'(Z[i][k])
__global__ void k_dense_xgrad(int B, int nin, int nout, const float *__restrict__ dY, const float *__restrict__ W,
                              const float *__restrict__ Zin, float *__restrict__ dX) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * nin) return;
    const int i = e / nin, k = e % nin;
    float s = 0.0f;
    for (int o = 0; o < nout; o++) s += dY[i * nout + o] * W[o * nin + k];
    dX[e] = Zin[e] > 0.0f ? s : 0.0f;
}

// loss = (1/B) sum_i sum_j w_j (out_ij - y_ij)^2 (partials per sample);
// dOut = (2/B) w_j (out - y)
__global__ void k_mse(int B, int nout, const float *__restrict__ out, const float *__restrict__ Y,
                      const float *__restrict__ wj, float *__restrict__ dOut, float *__restrict__ lpart) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    float l = 0.0f;
    for (int j = 0; j < nout; j++) {
        const float d = out[i * nout + j] - Y[i * nout + j];
        l += wj[j] * d * d;
        dOut[i * nout + j] = 2.0f * wj[j] * d / (float)B;
    }
    lpart[i] = l / (float)B;
}

__global__ void k_sum(int n, const float *__restrict__ a, float *__restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float s = 0.0f;
        for (int i = 0; i < n; i++) s += a[i];
        *out = s;
    }
}

// Adam (Kingma & Ba 2015), bias-corrected, with decoupled weight decay wd
// (AdamW, Loshchilov & Hutter 2019), on the flat parameter array
__global__ void k_adam(int n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2, float wd) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * p[e]);
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// activations workspace: Z and Y for the 4 layers (B x dims)
struct Acts {
    float *Z[NL], *Y[NL];
};

fd_status forward(const float *P, int B, const float *X, Acts &a, hipStream_t s) {
    const float *in = X;
    for (int l = 0; l < NL; l++) {
        const float *W = P + w_off(l);
        const float *b = W + (int64_t)DIMS[l + 1] * DIMS[l];
        hipLaunchKernelGGL(k_dense_fwd, dim3(nblk((int64_t)B * DIMS[l + 1])), dim3(256), 0, s, B, DIMS[l],
                           DIMS[l + 1], in, W, b, a.Z[l], a.Y[l], l < NL - 1 ? 1 : 0);
        FD_HIP(hipGetLastError());
        in = a.Y[l];
    }
    return FD_OK;
}

fd_status acts_alloc(int B, Acts &a, float **extra, int64_t extra_n) {
    int64_t tot = 0;
    for (int l = 0; l < NL; l++) tot += 2 * (int64_t)B * DIMS[l + 1];
    tot += extra_n;
    float *w = (float *)workspace(tot * sizeof(float), 6);
    if (!w) return fail(FD_ERR_OOM, "mlp: workspace");
    for (int l = 0; l < NL; l++) {
        a.Z[l] = w;
        w += (int64_t)B * DIMS[l + 1];
        a.Y[l] = w;
        w += (int64_t)B * DIMS[l + 1];
    }
    *extra = w;
    return FD_OK;
}

}  // namespace

fd_status mlp_forward(const float *P, int B, const float *X, float *out, hipStream_t s) {
    if (!P || !X || !out || B < 1 || B > 65536) return fail(FD_ERR_INVALID, "mlp_forward: bad arguments");
    Acts a;
    float *extra;
    FD_TRY(acts_alloc(B, a, &extra, 0));
    FD_TRY(forward(P, B, X, a, s));
    FD_HIP(hipMemcpyAsync(out, a.Y[NL - 1], (size_t)B * FD_MLP_OUT * sizeof(float), hipMemcpyDeviceToDevice, s));
    return FD_OK;
}

fd_status mlp_grad(const float *P, int B, const float *X, const float *Y, const float *wj, float *G,
                   float *loss_dev, hipStream_t s) {
    if (!P || !X || !Y || !wj || !G || B < 1 || B > 65536) return fail(FD_ERR_INVALID, "mlp_grad: bad arguments");
    Acts a;
    float *extra;
    // extra: dOut / dX ping-pong (2 x B x hidden) + loss partials (B)
    FD_TRY(acts_alloc(B, a, &extra, 2 * (int64_t)B * FD_MLP_HIDDEN + B));
    float *d0 = extra, *d1 = extra + (int64_t)B * FD_MLP_HIDDEN, *lp = d1 + (int64_t)B * FD_MLP_HIDDEN;
    FD_TRY(forward(P, B, X, a, s));
    hipLaunchKernelGGL(k_mse, dim3(nblk(B)), dim3(256), 0, s, B, FD_MLP_OUT, a.Y[NL - 1], Y, wj, d0, lp);
    FD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, B, lp, loss_dev);
    FD_HIP(hipGetLastError());
    for (int l = NL - 1; l >= 0; l--) {
        const float *in = l == 0 ? X : a.Y[l - 1];
        float *dW = G + w_off(l);
        float *db = dW + (int64_t)DIMS[l + 1] * DIMS[l];
        hipLaunchKernelGGL(k_dense_wgrad, dim3(nblk((int64_t)DIMS[l + 1] * (DIMS[l] + 1))), dim3(256), 0, s, B,
                           DIMS[l], DIMS[l + 1], in, d0, dW, db);
        FD_HIP(hipGetLastError());
        if (l > 0) {
            const float *W = P + w_off(l);
            hipLaunchKernelGGL(k_dense_xgrad, dim3(nblk((int64_t)B * DIMS[l])), dim3(256), 0, s, B, DIMS[l],
                               DIMS[l + 1], d0, W, a.Z[l - 1], d1);
            FD_HIP(hipGetLastError());
            std::swap(d0, d1);
        }
    }
    return FD_OK;
}

fd_status mlp_adam(float *P, const float *G, float *M, float *V, int step, float lr, float wd, hipStream_t s) {
    if (!P || !G || !M || !V || step < 1 || !(lr > 0) || !(wd >= 0)) return fail(FD_ERR_INVALID, "mlp_adam: bad arguments");
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(FD_MLP_NPARAMS)), dim3(256), 0, s, (int)FD_MLP_NPARAMS, P, G, M, V, lr, b1,
                       b2, 1e-8f, c1, c2, wd);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

}  // namespace fd
