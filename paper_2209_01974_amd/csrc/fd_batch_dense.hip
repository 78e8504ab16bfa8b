// Dense steps of the batched FD on gfx950, all instances per launch: for
// search spaces of n <= 64 vectors per instance the Gram products, the
// rotations, the residual norms, the Cholesky inverse and the symmetric
// eigensolve of every instance run as one launch each, instead of one chain
// of small launches per instance.  Instance i owns rows [off[i], off[i+1])
// of the row-major blocks (leading dimension ld); its n x n matrices sit at
// i n^2 of the small arrays.  A mask (device, per instance) skips instances
// that are done.  Reductions go slice by slice in a fixed order, so results
// do not depend on timing.
#include "fd_internal.h"

namespace fd {
namespace {

constexpr int NMAX = 64;

// Partial Gram of one slice of rows: P[slice] = X[r0:r1]^t Y[r0:r1] (n x n).
__global__ __launch_bounds__(256) void k_seg_gram_part(int n, const double *__restrict__ X,
                                                       const double *__restrict__ Y, int64_t ld,
                                                       const int32_t *__restrict__ seg_inst,
                                                       const int64_t *__restrict__ seg_r0,
                                                       const int64_t *__restrict__ seg_r1,
                                                       const int32_t *__restrict__ mask, double *__restrict__ P) {
    const int sg = blockIdx.x;
    const int i = seg_inst[sg];
    if (mask && !mask[i]) return;
    const int64_t r0 = seg_r0[sg], r1 = seg_r1[sg];
    __shared__ double xs[32][NMAX + 1], ys[32][NMAX + 1];
    const int t = threadIdx.x;
    const int ta = t / 16, tb = t % 16;  // 4 x 4 outputs each: rows ta*4.., cols tb*4..
    double acc[4][4] = {};
    for (int64_t rr = r0; rr < r1; rr += 32) {
        for (int e = t; e < 32 * NMAX; e += 256) {
            const int k = e / NMAX, c = e % NMAX;
            const int64_t r = rr + k;
            const bool ok = r < r1 && c < n;
            xs[k][c] = ok ? X[r * ld + c] : 0.0;
            ys[k][c] = ok ? Y[r * ld + c] : 0.0;
        }
        __syncthreads();
        for (int k = 0; k < 32; k++) {
            double xa[4], yb[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                xa[u] = xs[k][ta * 4 + u];
                yb[u] = ys[k][tb * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int v = 0; v < 4; v++) acc[u][v] += xa[u] * yb[v];
        }
        __syncthreads();
    }
    double *out = P + (int64_t)sg * n * n;
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int a = ta * 4 + u, b = tb * 4 + v;
            if (a < n && b < n) out[a * n + b] = acc[u][v];
        }
}

// G[i] = sum of the slices of instance i, in slice order.
__global__ __launch_bounds__(256) void k_seg_sum(int len, const double *__restrict__ P,
                                                 const int32_t *__restrict__ inst_s0,
                                                 const int32_t *__restrict__ mask, double *__restrict__ G) {
    const int i = blockIdx.x;
    if (mask && !mask[i]) return;
    const int s0 = inst_s0[i], s1 = inst_s0[i + 1];
    for (int e = threadIdx.x; e < len; e += 256) {
        double s = 0.0;
        for (int sg = s0; sg < s1; sg++) s += P[(int64_t)sg * len + e];
        G[(int64_t)i * len + e] = s;
    }
}

constexpr int RCH = 32;  // rows per rotation chunk

// X[r0:r1] <- X[r0:r1] Q[i] in place (a chunk of <= RCH rows of instance i).
__global__ __launch_bounds__(256) void k_seg_rotate(int n, double *__restrict__ X, int64_t ld,
                                                    const double *__restrict__ Q,
                                                    const int32_t *__restrict__ rc_inst,
                                                    const int64_t *__restrict__ rc_r0,
                                                    const int64_t *__restrict__ off,
                                                    const int32_t *__restrict__ mask) {
    const int c = blockIdx.x;
    const int i = rc_inst[c];
    if (mask && !mask[i]) return;
    const int64_t r0 = rc_r0[c], r1 = min(r0 + RCH, off[i + 1]);
    const int nr = (int)(r1 - r0);
    __shared__ double q[NMAX][NMAX + 1], xr[RCH][NMAX + 1];
    const double *Qi = Q + (int64_t)i * n * n;
    for (int e = threadIdx.x; e < n * n; e += 256) q[e / n][e % n] = Qi[e];
    for (int e = threadIdx.x; e < RCH * n; e += 256) {
        const int r = e / n, k = e % n;
        xr[r][k] = r < nr ? X[(r0 + r) * ld + k] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x / 8, g = threadIdx.x % 8;
    if (r >= nr) return;
    for (int j = g; j < n; j += 8) {
        double s = 0.0;
        for (int k = 0; k < n; k++) s += xr[r][k] * q[k][j];
        X[(r0 + r) * ld + j] = s;
    }
}

// Partial residual sums of a slice: P[slice][j] = sum_r (W[r][j] - theta_j V[r][j])^2.
__global__ __launch_bounds__(256) void k_seg_resid_part(int n, const double *__restrict__ V,
                                                        const double *__restrict__ W, int64_t ld,
                                                        const double *__restrict__ theta,
                                                        const int32_t *__restrict__ seg_inst,
                                                        const int64_t *__restrict__ seg_r0,
                                                        const int64_t *__restrict__ seg_r1,
                                                        const int32_t *__restrict__ mask, double *__restrict__ P) {
    const int sg = blockIdx.x;
    const int i = seg_inst[sg];
    if (mask && !mask[i]) return;
    const int64_t r0 = seg_r0[sg], r1 = seg_r1[sg];
    __shared__ double part[4][NMAX];
    const int j = threadIdx.x % NMAX, lane = threadIdx.x / NMAX;
    double s = 0.0;
    if (j < n) {
        const double th = theta[(int64_t)i * n + j];
        for (int64_t r = r0 + lane; r < r1; r += 4) {
            const double e = W[r * ld + j] - th * V[r * ld + j];
            s += e * e;
        }
    }
    part[lane][j] = s;
    __syncthreads();
    if (lane == 0 && j < n) P[(int64_t)sg * n + j] = ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j];
}

__global__ void k_sqrt_b(int64_t len, double *x) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) x[e] = sqrt(x[e]);
}

__global__ void k_sym_b(int n_inst, int n, double *G) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n_inst * n * n) return;
    const int64_t i = e / ((int64_t)n * n);
    const int loc = (int)(e - i * n * n);
    const int a = loc / n, b = loc % n;
    if (a < b) {
        double *g = G + i * n * n;
        const double v = 0.5 * (g[a * n + b] + g[b * n + a]);
        g[a * n + b] = v;
        g[b * n + a] = v;
    }
}

// G = R^t R (R upper), then Q = R^-1, per instance; ok[i] = 0 if a pivot
// falls to 1e-14 n of its own diagonal entry or below, or (near_identity,
// the second CholQR pass) if an entry of G is more than 0.5 from the
// identity.
__global__ __launch_bounds__(256) void k_cholinv_b(int n, double *__restrict__ Gall, double *__restrict__ Qall,
                                                   int32_t *__restrict__ ok, const int32_t *__restrict__ mask,
                                                   int near_identity) {
    const int i = blockIdx.x;
    if (mask && !mask[i]) return;
    double *G = Gall + (int64_t)i * n * n, *Q = Qall + (int64_t)i * n * n;
    __shared__ int good;
    __shared__ double d0[NMAX];
    if (threadIdx.x == 0) good = 1;
    for (int k = threadIdx.x; k < n; k += blockDim.x) d0[k] = G[k * n + k];
    __syncthreads();
    if (near_identity) {
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            const double dev = G[e] - ((e / n == e % n) ? 1.0 : 0.0);
            if (!(fabs(dev) <= 0.5)) good = 0;
        }
        __syncthreads();
        if (!good) {
            if (threadIdx.x == 0) ok[i] = 0;
            return;
        }
    }
    const double rel = 1e-14 * (double)n;
    for (int k = 0; k < n; k++) {
        const double piv = G[k * n + k];
        if (!(piv > rel * d0[k])) {
            if (threadIdx.x == 0) good = 0;
            break;
        }
        const double r = sqrt(piv);
        __syncthreads();
        for (int j = k + threadIdx.x; j < n; j += blockDim.x) G[k * n + j] = (j == k) ? r : G[k * n + j] / r;
        __syncthreads();
        const int rem = n - k - 1;
        for (int e = threadIdx.x; e < rem * rem; e += blockDim.x) {
            const int a = k + 1 + e / rem, b = k + 1 + e % rem;
            if (b >= a) G[a * n + b] -= G[k * n + a] * G[k * n + b];
        }
        __syncthreads();
    }
    __syncthreads();
    if (!good) {
        if (threadIdx.x == 0) ok[i] = 0;
        return;
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        for (int a = n - 1; a >= 0; a--) {
            double s = (a == j) ? 1.0 : 0.0;
            if (a > j) {
                Q[a * n + j] = 0.0;
                continue;
            }
            for (int k = a + 1; k <= j; k++) s -= G[a * n + k] * Q[k * n + j];
            Q[a * n + j] = s / G[a * n + a];
        }
    }
    if (threadIdx.x == 0) ok[i] = 1;
}

// Symmetric eigensolve of one n x n matrix per block (n <= 64): cyclic
// Jacobi with the round-robin (tournament) ordering, n/2 disjoint rotations
// per step, in LDS.  A rotation of the pair (p, q) zeroes A[p][q]
// (t = sign(th) / (|th| + sqrt(th^2 + 1)), th = (a_qq - a_pp) / (2 a_pq));
// it is skipped when |a_pq| <= 1e-18 sqrt(|a_pp a_qq|).  Sweeps stop when
// the off-diagonal Frobenius norm is <= 1e-13 of the whole (at most 40).
// Output: eigenvalues ascending in w[i n ..], eigenvectors as the columns of
// U[i] (row-major, U[k][j] = component k of vector j).
__global__ __launch_bounds__(256) void k_jacobi_b(int n, const double *__restrict__ S, double *__restrict__ w,
                                                  double *__restrict__ U, const int32_t *__restrict__ mask) {
    const int i = blockIdx.x;
    if (mask && !mask[i]) return;
    const int m = n + (n & 1);
    const int np = m / 2;
    // A and the vectors in dynamic LDS (2 x 64 x 65 doubles, over the 64 KB
    // of static LDS; the launch raises the limit)
    extern __shared__ double dyn[];
    double(*A)[NMAX + 1] = reinterpret_cast<double(*)[NMAX + 1]>(dyn);
    double(*Vm)[NMAX + 1] = reinterpret_cast<double(*)[NMAX + 1]>(dyn + NMAX * (NMAX + 1));
    __shared__ double cs[NMAX / 2], sn[NMAX / 2];
    __shared__ int pp[NMAX / 2], qq[NMAX / 2], pl[NMAX];
    __shared__ double red[256];
    __shared__ int stop;
    const int t = threadIdx.x;
    const double *Si = S + (int64_t)i * n * n;
    for (int e = t; e < m * m; e += 256) {
        const int a = e / m, b = e % m;
        A[a][b] = (a < n && b < n) ? Si[a * n + b] : 0.0;
        Vm[a][b] = (a == b) ? 1.0 : 0.0;
    }
    if (t < m) pl[t] = t;
    __syncthreads();
    // squared Frobenius norm of A
    double s2 = 0.0;
    for (int e = t; e < m * m; e += 256) s2 += A[e / m][e % m] * A[e / m][e % m];
    red[t] = s2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double nrm2 = red[0];
    __syncthreads();
    for (int sweep = 0; sweep < 40; sweep++) {
        double o2 = 0.0;
        for (int e = t; e < m * m; e += 256) {
            const int a = e / m, b = e % m;
            if (a != b) o2 += A[a][b] * A[a][b];
        }
        red[t] = o2;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        if (t == 0) stop = red[0] <= 1e-26 * nrm2;
        __syncthreads();
        if (stop) break;
        for (int step = 0; step < m - 1; step++) {
            if (t < np) {
                int p = pl[t], q = pl[m - 1 - t];
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq))) {
                    const double th = (aqq - app) / (2.0 * apq);
                    double tt;
                    if (fabs(th) < 1e150) tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    else tt = 0.5 / th;
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                }
                pp[t] = p;
                qq[t] = q;
                cs[t] = c;
                sn[t] = s;
            }
            __syncthreads();
            // rows p and q of every pair
            for (int e = t; e < np * m; e += 256) {
                const int k = e / m, col = e % m;
                const int p = pp[k], q = qq[k];
                const double c = cs[k], s = sn[k];
                const double ap = A[p][col], aq = A[q][col];
                A[p][col] = c * ap - s * aq;
                A[q][col] = s * ap + c * aq;
            }
            __syncthreads();
            // columns p and q of every pair, and of the vectors
            for (int e = t; e < np * m; e += 256) {
                const int k = e / m, row = e % m;
                const int p = pp[k], q = qq[k];
                const double c = cs[k], s = sn[k];
                const double ap = A[row][p], aq = A[row][q];
                A[row][p] = c * ap - s * aq;
                A[row][q] = s * ap + c * aq;
                const double vp = Vm[row][p], vq = Vm[row][q];
                Vm[row][p] = c * vp - s * vq;
                Vm[row][q] = s * vp + c * vq;
            }
            __syncthreads();
            // next round-robin pairing (position 0 stays)
            if (t == 0) {
                const int tmp = pl[m - 1];
                for (int k = m - 1; k > 1; k--) pl[k] = pl[k - 1];
                pl[1] = tmp;
            }
            __syncthreads();
        }
    }
    // ascending order (ties by index); only the first n (the padding of an
    // odd n never mixes with them)
    if (t < n) {
        const double v = A[t][t];
        int rank = 0;
        for (int k = 0; k < n; k++) {
            const double u = A[k][k];
            rank += (u < v) || (u == v && k < t);
        }
        w[(int64_t)i * n + rank] = v;
        double *Ui = U + (int64_t)i * n * n;
        for (int row = 0; row < n; row++) Ui[row * n + rank] = Vm[row][t];
    }
}

// SVQB (Stathopoulos & Wu 2002), per instance: d = diag(G)^-1/2 (1 for a
// zero column), G <- D G D.
__global__ __launch_bounds__(256) void k_svqb_prep_b(int n, double *__restrict__ Gall, double *__restrict__ dall,
                                                     const int32_t *__restrict__ mask) {
    const int i = blockIdx.x;
    if (mask && !mask[i]) return;
    double *G = Gall + (int64_t)i * n * n, *d = dall + (int64_t)i * n;
    for (int k = threadIdx.x; k < n; k += 256) {
        const double g = G[k * n + k];
        d[k] = (g > 0.0) ? 1.0 / sqrt(g) : 1.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += 256) G[e] *= d[e / n] * d[e % n];
}

// Q = D U L^-1/2 with L clipped at 1e-14 max(L); rank[i] = unclipped count.
__global__ __launch_bounds__(256) void k_svqb_q_b(int n, const double *__restrict__ dall,
                                                  const double *__restrict__ lall, const double *__restrict__ Uall,
                                                  double *__restrict__ Qall, int32_t *__restrict__ rank,
                                                  const int32_t *__restrict__ mask) {
    const int i = blockIdx.x;
    if (mask && !mask[i]) return;
    const double *d = dall + (int64_t)i * n, *lam = lall + (int64_t)i * n, *U = Uall + (int64_t)i * n * n;
    double *Q = Qall + (int64_t)i * n * n;
    __shared__ double fl;
    __shared__ int cnt;
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int j = 0; j < n; j++) mx = fmax(mx, lam[j]);
        fl = 1e-14 * mx;
        int c = 0;
        for (int j = 0; j < n; j++) c += (lam[j] > fl && fl > 0.0);
        cnt = c;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += 256) {
        const int a = e / n, j = e % n;
        const double l = fmax(lam[j], fl > 0.0 ? fl : 1.0);
        Q[e] = d[a] * U[e] / sqrt(l);
    }
    if (threadIdx.x == 0) rank[i] = cnt;
}

}  // namespace

fd_status batched_svqb(int n_inst, int n, double *G, double *d, double *lam, double *U, double *Q, int32_t *rank,
                       const int32_t *mask, hipStream_t s) {
    if (n < 1 || n > NMAX) return fail(FD_ERR_INVALID, "batched SVQB: n must be in [1, 64]");
    hipLaunchKernelGGL(k_svqb_prep_b, dim3(n_inst), dim3(256), 0, s, n, G, d, mask);
    FD_HIP(hipGetLastError());
    FD_TRY(batched_syev(n_inst, n, G, lam, U, mask, s));
    hipLaunchKernelGGL(k_svqb_q_b, dim3(n_inst), dim3(256), 0, s, n, d, lam, U, Q, rank, mask);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status seg_gram(const BatchDev &B, int n, const double *X, const double *Y, int64_t ld, const int32_t *mask,
                   double *P, double *G, hipStream_t s) {
    if (n < 1 || n > NMAX) return fail(FD_ERR_INVALID, "batched Gram: n must be in [1, 64]");
    hipLaunchKernelGGL(k_seg_gram_part, dim3(B.nseg), dim3(256), 0, s, n, X, Y, ld, B.seg_inst, B.seg_r0, B.seg_r1,
                       mask, P);
    FD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_seg_sum, dim3(B.n_inst), dim3(256), 0, s, n * n, P, B.inst_s0, mask, G);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status seg_rotate(const BatchDev &B, int n, double *X, int64_t ld, const double *Q, const int32_t *mask,
                     hipStream_t s) {
    if (n < 1 || n > NMAX) return fail(FD_ERR_INVALID, "batched rotation: n must be in [1, 64]");
    hipLaunchKernelGGL(k_seg_rotate, dim3(B.nrc), dim3(256), 0, s, n, X, ld, Q, B.rc_inst, B.rc_r0, B.off, mask);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status seg_resid(const BatchDev &B, int n, const double *V, const double *W, int64_t ld, const double *theta,
                    const int32_t *mask, double *P, double *rho, hipStream_t s) {
    if (n < 1 || n > NMAX) return fail(FD_ERR_INVALID, "batched residuals: n must be in [1, 64]");
    hipLaunchKernelGGL(k_seg_resid_part, dim3(B.nseg), dim3(256), 0, s, n, V, W, ld, theta, B.seg_inst, B.seg_r0,
                       B.seg_r1, mask, P);
    FD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_seg_sum, dim3(B.n_inst), dim3(256), 0, s, n, P, B.inst_s0, mask, rho);
    FD_HIP(hipGetLastError());
    const int64_t len = (int64_t)B.n_inst * n;
    hipLaunchKernelGGL(k_sqrt_b, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, len, rho);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status batched_sym(int n_inst, int n, double *G, hipStream_t s) {
    const int64_t len = (int64_t)n_inst * n * n;
    hipLaunchKernelGGL(k_sym_b, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, n_inst, n, G);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status batched_cholinv(int n_inst, int n, double *G, double *Q, int32_t *ok, const int32_t *mask,
                          bool second_pass, hipStream_t s) {
    if (n < 1 || n > NMAX) return fail(FD_ERR_INVALID, "batched Cholesky: n must be in [1, 64]");
    hipLaunchKernelGGL(k_cholinv_b, dim3(n_inst), dim3(256), 0, s, n, G, Q, ok, mask, second_pass ? 1 : 0);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status batched_syev(int n_inst, int n, const double *S, double *w, double *U, const int32_t *mask, hipStream_t s) {
    if (n < 1 || n > NMAX) return fail(FD_ERR_INVALID, "batched eigensolve: n must be in [1, 64]");
    const size_t sh = 2 * NMAX * (NMAX + 1) * sizeof(double);
    FD_HIP(hipFuncSetAttribute((const void *)k_jacobi_b, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
    hipLaunchKernelGGL(k_jacobi_b, dim3(n_inst), dim3(256), sh, s, n, S, w, U, mask);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

}  // namespace fd
