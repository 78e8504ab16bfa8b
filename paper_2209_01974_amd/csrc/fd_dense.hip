// Dense FP64 kernels for the orthogonalization and Rayleigh-Ritz steps on
// gfx950.
//
// Sec. 2 / Sec. 3: after each filter application the N_s search vectors are
// orthogonalized (SVQB needs only the N_s x N_s Gram matrix V^t V), and one
// more SpMV gives the Ritz values.  Both reduce to tall-skinny products over
// D rows (X^t Y and X Q) -- dense contractions, done here on the FP64 matrix
// cores with v_mfma_f64_16x16x4_f64 -- plus work on N_s x N_s matrices that
// runs inside one workgroup (parallel cyclic Jacobi, Cholesky, triangular
// inverse).  Reductions over D are two-stage with a fixed order, so repeated
// runs are bitwise identical.
#include <cmath>
#include <mutex>
#include <vector>

#include "fd_internal.h"

namespace fd {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// MFMA f64 16x16x4 operand layout (lane l = i + 16 k):
//   A[i][k] (16 x 4) and B[k][j] (4 x 16) hold one double per lane;
//   the 16 x 16 result keeps D[(l >> 4) + 4 r][l & 15] in element r.
__device__ __forceinline__ dbl4 mfma16x16x4(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------ workspace --
namespace {
struct WsSlot {
    void *p = nullptr;
    size_t n = 0;
    int dev = -1;
};
std::mutex g_ws_mu;
WsSlot g_ws[10];
}  // namespace

void *workspace(size_t bytes, int slot) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    WsSlot &w = g_ws[slot];
    if (w.p && w.n >= bytes && w.dev == dev) return w.p;
    if (w.p) {
        (void)hipDeviceSynchronize();
        (void)hipFree(w.p);
        w.p = nullptr;
        w.n = 0;
    }
    size_t want = std::max<size_t>(bytes, 1 << 20);
    if (hipMalloc(&w.p, want) != hipSuccess) {
        w.p = nullptr;
        return nullptr;
    }
    w.n = want;
    w.dev = dev;
    return w.p;
}

// ----------------------------------------------------------------- Gram --
namespace {

constexpr int GT = 64;  // Gram tile edge per wave

struct TileList {
    int n;
    unsigned char ti[64], tj[64];
};

__global__ __launch_bounds__(64) void k_gram(const double *__restrict__ X, int64_t ldx,
                                              const double *__restrict__ Y, int64_t ldy,
                                              int64_t D, int m, int n, int64_t rps, TileList tl,
                                              double *__restrict__ P) {
    const int tile = blockIdx.x;
    const int64_t slice = blockIdx.y;
    const int ti = tl.ti[tile], tj = tl.tj[tile];
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int64_t r0 = slice * rps;
    const int64_t r1 = min(D, r0 + rps);
    dbl4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = (dbl4)0.0;
    int ca[4], cb[4];
    bool va[4], vb[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        ca[q] = ti * GT + q * 16 + li;
        cb[q] = tj * GT + q * 16 + li;
        va[q] = ca[q] < m;
        vb[q] = cb[q] < n;
    }
    for (int64_t r = r0; r < r1; r += 4) {
        const int64_t rr = r + lk;
        const bool rv = rr < r1;
        double a[4], b[4];
        const double *xr = X + rr * ldx;
        const double *yr = Y + rr * ldy;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            a[q] = (rv && va[q]) ? xr[ca[q]] : 0.0;
            b[q] = (rv && vb[q]) ? yr[cb[q]] : 0.0;
        }
#pragma unroll
        for (int qa = 0; qa < 4; qa++)
#pragma unroll
            for (int qb = 0; qb < 4; qb++) acc[qa][qb] = mfma16x16x4(a[qa], b[qb], acc[qa][qb]);
    }
    double *out = P + ((int64_t)slice * tl.n + tile) * (GT * GT);
#pragma unroll
    for (int qa = 0; qa < 4; qa++)
#pragma unroll
        for (int qb = 0; qb < 4; qb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int il = qa * 16 + (lane >> 4) + 4 * r;
                const int jl = qb * 16 + (lane & 15);
                out[il * GT + jl] = acc[qa][qb][r];
            }
}

__global__ void k_gram_reduce(const double *__restrict__ P, int S, int ntiles, int m, int n,
                              bool sym, int nt_n, int te, double *__restrict__ G, int64_t ldg) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * n) return;
    int i = (int)(e / n), j = (int)(e % n);
    if (sym && i > j) {
        int t = i;
        i = j;
        j = t;
    }
    const int ti = i / te, tj = j / te;
    int tile;
    if (sym) {
        // upper-triangle tiles listed row by row: (0,0..T-1), (1,1..T-1), ...
        tile = ti * nt_n - ti * (ti - 1) / 2 + (tj - ti);
    } else {
        tile = ti * nt_n + tj;
    }
    const int64_t tsz = (int64_t)te * te;
    const int64_t off = (int64_t)tile * tsz + (i % te) * te + (j % te);
    double s = 0.0;
    for (int k = 0; k < S; k++) s += P[(int64_t)k * ntiles * tsz + off];
    G[(e / n) * ldg + (e % n)] = s;
}

// Gram products with both sides at least 128 wide: a block of 4 waves owns
// a 128 x 128 tile of the result (a 64 x 64 quarter per wave) over a slice
// of rows.  The rows of the tile's 128 + 128 columns go through LDS in
// chunks of 16, so that each value loaded from memory feeds two waves'
// matrix cores; the next chunk is loaded into registers while the current
// one is multiplied.
constexpr int GB = 128;      // block tile edge
constexpr int GK = 16;        // rows per chunk
constexpr int GLD = GB + 16; // LDS row stride (doubles): alternate rows on the two bank halves

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gram_big(const double *__restrict__ X, int64_t ldx,
                                                  const double *__restrict__ Y, int64_t ldy, int64_t D,
                                                  int m, int n, int64_t rps, TileList tl,
                                                  double *__restrict__ P) {
    __shared__ double sA[GK * GLD];
    __shared__ double sB[GK * GLD];
    const int tile = blockIdx.x;
    const int64_t slice = blockIdx.y;
    const int ti = tl.ti[tile], tj = tl.tj[tile];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
    const int wi = wave >> 1, wj = wave & 1;
    const int64_t r0 = slice * rps;
    const int64_t r1 = min(D, r0 + rps);
    // staging map: element u of a thread is row (u * 256 + t) / 128, column
    // (u * 256 + t) % 128 of the chunk: 8 per operand, coalesced along rows
    const int scol = t & (GB - 1), srow = t >> 7;  // srow in {0, 1}
    const int ca = ti * GB + scol, cb = tj * GB + scol;
    const bool va = ca < m, vb = cb < n;
    double ra[GK / 2], rb[GK / 2];
    auto fetch = [&](int64_t c0) {
#pragma unroll
        for (int u = 0; u < GK / 2; u++) {
            const int64_t r = c0 + 2 * u + srow;
            const bool rv = r < r1;
            ra[u] = (rv && va) ? X[r * ldx + ca] : 0.0;
            rb[u] = (rv && vb) ? Y[r * ldy + cb] : 0.0;
        }
    };
    dbl4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = (dbl4)0.0;
    fetch(r0);
    for (int64_t c0 = r0; c0 < r1; c0 += GK) {
        __syncthreads();  // the previous chunk is no longer read
#pragma unroll
        for (int u = 0; u < GK / 2; u++) {
            sA[(2 * u + srow) * GLD + scol] = ra[u];
            sB[(2 * u + srow) * GLD + scol] = rb[u];
        }
        __syncthreads();
        if (c0 + GK < r1) fetch(c0 + GK);
#pragma unroll
        for (int ks = 0; ks < GK / 4; ks++) {
            const int k = ks * 4 + lk;
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                a[q] = sA[k * GLD + wi * 64 + q * 16 + li];
                b[q] = sB[k * GLD + wj * 64 + q * 16 + li];
            }
#pragma unroll
            for (int qa = 0; qa < 4; qa++)
#pragma unroll
                for (int qb = 0; qb < 4; qb++) acc[qa][qb] = mfma16x16x4(a[qa], b[qb], acc[qa][qb]);
        }
    }
    double *out = P + ((int64_t)slice * tl.n + tile) * (GB * GB);
#pragma unroll
    for (int qa = 0; qa < 4; qa++)
#pragma unroll
        for (int qb = 0; qb < 4; qb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int il = wi * 64 + qa * 16 + (lane >> 4) + 4 * r;
                const int jl = wj * 64 + qb * 16 + (lane & 15);
                out[il * GB + jl] = acc[qa][qb][r];
            }
}

}  // namespace

fd_status gram(int64_t D, int m, int n, const double *X, int64_t ldx, const double *Y,
               int64_t ldy, double *G, int64_t ldg, bool sym, hipStream_t s) {
    if (m < 1 || n < 1 || m > 512 || n > 512 || D < 1)
        return fail(FD_ERR_INVALID, "gram: need 1 <= m, n <= 512 and D >= 1");
    if (sym && m != n) return fail(FD_ERR_INVALID, "gram: symmetric product needs m == n");
    const bool big = m >= GB && n >= GB;
    const int te = big ? GB : GT;
    const int ntm = (m + te - 1) / te, ntn = (n + te - 1) / te;
    TileList tl;
    tl.n = 0;
    for (int a = 0; a < ntm; a++)
        for (int b = sym ? a : 0; b < ntn; b++) {
            tl.ti[tl.n] = (unsigned char)a;
            tl.tj[tl.n] = (unsigned char)b;
            tl.n++;
        }
    // slices of rows: about 2048 waves in all (512 blocks of 4 for big tiles)
    int64_t target = std::max<int64_t>(1, (big ? 512 : 2048) / tl.n);
    int64_t rps = std::max<int64_t>(256, (D + target - 1) / target);
    rps = (rps + GK - 1) / GK * GK;
    int64_t S = (D + rps - 1) / rps;
    double *P = (double *)workspace((size_t)S * tl.n * te * te * sizeof(double), 0);
    if (!P) return fail(FD_ERR_OOM, "gram: workspace");
    if (big)
        hipLaunchKernelGGL(k_gram_big, dim3(tl.n, (unsigned)S), dim3(256), 0, s, X, ldx, Y, ldy, D, m, n, rps,
                           tl, P);
    else
        hipLaunchKernelGGL(k_gram, dim3(tl.n, (unsigned)S), dim3(64), 0, s, X, ldx, Y, ldy, D, m, n, rps,
                           tl, P);
    FD_HIP(hipGetLastError());
    const int64_t tot = (int64_t)m * n;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, P, (int)S,
                       tl.n, m, n, sym, ntn, te, G, ldg);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

// ------------------------------------------------------------- rotation --
namespace {

template <int TM>
__global__ __launch_bounds__(512) void k_rotate(double *__restrict__ X, int64_t ldx, int64_t D,
                                                 int m, int n, const double *__restrict__ Q,
                                                 int64_t ldq, int ls, int g) {
    extern __shared__ double sX[];
    const int64_t r0 = (int64_t)blockIdx.x * TM;
    const int m4 = (m + 3) & ~3;
    // stage the row tile in LDS, 16 loads per thread in flight at a time
    const int tot = TM * m4;
    for (int base = 0; base < tot; base += 16 * 512) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int e = base + u * 512 + (int)threadIdx.x;
            double x = 0.0;
            if (e < tot) {
                const int r = e / m4, k = e - r * m4;
                const int64_t rr = r0 + r;
                if (rr < D && k < m) x = X[rr * ldx + k];
            }
            v[u] = x;
        }
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int e = base + u * 512 + (int)threadIdx.x;
            if (e < tot) {
                const int r = e / m4;
                sX[r * ls + (e - r * m4)] = v[u];
            }
        }
    }
    __syncthreads();
    constexpr int RB = TM / 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int ncb = (n + 15) >> 4;
    const int cb0 = wave * g;
    if (cb0 >= ncb) return;
    dbl4 acc[RB][4];
#pragma unroll
    for (int a = 0; a < RB; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = (dbl4)0.0;
    int cc[4];
    bool cv[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        cc[q] = (cb0 + q) * 16 + li;
        cv[q] = (q < g) && (cc[q] < n);
    }
    // Q streams from L2 for every row tile: the next k-step's entries are
    // loaded while the matrix cores work on the current ones
    double b[4], bn[4];
#pragma unroll
    for (int q = 0; q < 4; q++) b[q] = (lk < m && cv[q]) ? Q[(int64_t)lk * ldq + cc[q]] : 0.0;
    for (int k0 = 0; k0 < m4; k0 += 4) {
        const int kk = k0 + lk, kn = kk + 4;
#pragma unroll
        for (int q = 0; q < 4; q++) bn[q] = (kn < m && cv[q]) ? Q[(int64_t)kn * ldq + cc[q]] : 0.0;
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
            const double a = sX[(rb * 16 + li) * ls + kk];
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (q < g) acc[rb][q] = mfma16x16x4(a, b[q], acc[rb][q]);
        }
#pragma unroll
        for (int q = 0; q < 4; q++) b[q] = bn[q];
    }
#pragma unroll
    for (int rb = 0; rb < RB; rb++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (q >= g) continue;
            const int col = (cb0 + q) * 16 + (lane & 15);
            if (col >= n) continue;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t row = r0 + rb * 16 + (lane >> 4) + 4 * r;
                if (row < D) X[row * ldx + col] = acc[rb][q][r];
            }
        }
}

}  // namespace

fd_status rotate(int64_t D, int m, int n, double *X, int64_t ldx, const double *Q, int64_t ldq,
                 hipStream_t s) {
    if (m < 1 || n < 1 || n > m || m > 512 || D < 1)
        return fail(FD_ERR_INVALID, "rotate: need 1 <= n <= m <= 512 and D >= 1");
    const int m4 = (m + 3) & ~3;
    const int ls = ((m4 + 31) / 32) * 32 + 4;  // padded LDS row: spreads the 16 rows over banks
    const int ncb = (n + 15) / 16;
    const int g = std::min(4, (ncb + 7) / 8);
    if (m <= 256) {
        size_t sh = (size_t)32 * ls * sizeof(double);
        FD_HIP(hipFuncSetAttribute((const void *)k_rotate<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)sh));
        hipLaunchKernelGGL(k_rotate<32>, dim3((unsigned)((D + 31) / 32)), dim3(512), sh, s, X, ldx, D, m, n,
                           Q, ldq, ls, g);
    } else {
        size_t sh = (size_t)16 * ls * sizeof(double);
        FD_HIP(hipFuncSetAttribute((const void *)k_rotate<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)sh));
        hipLaunchKernelGGL(k_rotate<16>, dim3((unsigned)((D + 15) / 16)), dim3(512), sh, s, X, ldx, D, m, n,
                           Q, ldq, ls, g);
    }
    FD_HIP(hipGetLastError());
    return FD_OK;
}

// -------------------------------------------------------- block Jacobi --
// Symmetric eigensolver for n <= 512 (FP64): cyclic block Jacobi.  Indices
// are cut into blocks of 16; a round pairs the blocks by the round-robin
// ("chess tournament") schedule.  For every pair (I, J) one workgroup
// applies a sweep of scalar cyclic Jacobi to the 32 x 32 matrix
// A[I u J, I u J] in LDS and keeps the accumulated rotation R; then A <- J^t A J and U <- U J
// for the block-diagonal J of all pairs, as independent 32 x 32 tiles
// R_a^t A_ab R_b and U_rb R_b on the FP64 matrix cores.  Sweeps repeat until
// the off-diagonal norm stops decreasing or falls below 4 n eps ||A||_F.
// Indices past n are zero rows and columns: they never mix with the others.
namespace {

constexpr int JB = 16;  // index block
constexpr int JG = 32;  // pair group: two index blocks

struct PairList {
    int n;
    unsigned char I[16], J[16];
};

__device__ __forceinline__ int grp_index(int l, int I, int J) { return l < JB ? I * JB + l : J * JB + (l - JB); }

// Jacobi sweeps of a pair group per outer round.  One sweep per round (the
// outer iteration then behaves as a cyclic Jacobi sweep over all index
// pairs, in blocks) costs fewer outer sweeps' worth of time than
// diagonalizing each group to convergence: at n = 128, 2.9 ms against 4.7 ms
// for a random matrix, the same for a nearly diagonal one.
constexpr int kBjInner = 1;

// One pair group: diagonalize S = A[I u J, I u J] (32 x 32, in LDS) by
// cyclic Jacobi with the round-robin pairing, at most max_inner sweeps, and
// write the accumulated rotation R.  A round rotates 16 disjoint index pairs
// at once; the two-sided update S <- J^t S J is done as 256 independent
// 2 x 2 blocks (one per thread), R <- R J as 512 column pairs, so a round
// needs two barriers.
__global__ __launch_bounds__(256) void k_bj_solve(int np, const double *__restrict__ A, PairList pl,
                                                  double *__restrict__ Rbuf, double thr2, int max_inner) {
    __shared__ double red[2][4];
    __shared__ double S[JG][JG + 1];
    __shared__ double R[JG][JG + 1];
    __shared__ double cc[JG / 2], ss[JG / 2];
    __shared__ int pp[JG / 2], pq[JG / 2];
    const int k = blockIdx.x, I = pl.I[k], J = pl.J[k];
    const int lane = threadIdx.x;  // 0..255
    for (int e = lane; e < JG * JG; e += 256) {
        const int r = e / JG, c = e % JG;
        S[r][c] = A[(int64_t)grp_index(r, I, J) * np + grp_index(c, I, J)];
        R[r][c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    // the 2 x 2 block of this thread: pair indices ba (rows), bb (columns)
    const int ba = lane / (JG / 2), bb = lane % (JG / 2);
    for (int sweep = 0; sweep < max_inner; sweep++) {
        double off = 0.0, dg = 0.0;
        for (int e = lane; e < JG * JG; e += 256) {
            const int r = e / JG, c = e % JG;
            const double v = S[r][c];
            if (r == c) dg += v * v;
            else off += v * v;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o, 64);
            dg += __shfl_xor(dg, o, 64);
        }
        if ((lane & 63) == 0) {
            red[0][lane >> 6] = off;
            red[1][lane >> 6] = dg;
        }
        __syncthreads();
        off = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        dg = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        __syncthreads();
        // thr2: squared relative target, about 1e-3 of the whole matrix's
        // off-diagonal level after the previous sweep (down to 1e-16)
        if (!(off > thr2 * (off + dg))) break;
        for (int rnd = 0; rnd < JG - 1; rnd++) {
            if (lane < JG / 2) {
                auto who = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + rnd) % (JG - 1); };
                int p = who(lane), q = who(JG - 1 - lane);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, s = 0.0;
                const double apq = S[p][q];
                if (apq != 0.0) {
                    const double th = (S[q][q] - S[p][p]) / (2.0 * apq);
                    const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                pp[lane] = p;
                pq[lane] = q;
                cc[lane] = c;
                ss[lane] = s;
            }
            __syncthreads();
            {
                // S block (rows p_a, q_a; columns p_b, q_b) <- J_a^t S J_b,
                // J = [[c, s], [-s, c]] on (p, q)
                const double ca = cc[ba], sa = ss[ba], cb = cc[bb], sb = ss[bb];
                if (sa != 0.0 || sb != 0.0) {
                    const int pa = pp[ba], qa = pq[ba], pb = pp[bb], qb = pq[bb];
                    const double x00 = S[pa][pb], x01 = S[pa][qb], x10 = S[qa][pb], x11 = S[qa][qb];
                    const double y00 = cb * x00 - sb * x01, y01 = sb * x00 + cb * x01;
                    const double y10 = cb * x10 - sb * x11, y11 = sb * x10 + cb * x11;
                    S[pa][pb] = ca * y00 - sa * y10;
                    S[qa][qb] = sa * y01 + ca * y11;
                    if (ba == bb) {  // the rotated-away entry is exactly zero
                        S[pa][qb] = 0.0;
                        S[qa][pb] = 0.0;
                    } else {
                        S[pa][qb] = ca * y01 - sa * y11;
                        S[qa][pb] = sa * y00 + ca * y10;
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 2; h++) {  // R <- R J: row i, pair kk
                const int e = lane + 256 * h, i = e / (JG / 2), kk = e % (JG / 2);
                const double s = ss[kk];
                if (s != 0.0) {
                    const int p = pp[kk], q = pq[kk];
                    const double c = cc[kk], rp = R[i][p], rq = R[i][q];
                    R[i][p] = c * rp - s * rq;
                    R[i][q] = s * rp + c * rq;
                }
            }
            __syncthreads();
        }
    }
    double *Ro = Rbuf + (int64_t)k * JG * JG;
    for (int e = lane; e < JG * JG; e += 256) Ro[e] = R[e / JG][e % JG];
}

// out = X * Y for 32 x 32 LDS tiles (TX: use X^t), one wavefront, FP64 MFMA.
template <bool TX>
__device__ void mm32(const double (*X)[JG + 1], const double (*Y)[JG + 1], double (*O)[JG + 1]) {
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = (dbl4)0.0;
#pragma unroll
    for (int k0 = 0; k0 < JG; k0 += 4) {
        double xa[2], yb[2];
#pragma unroll
        for (int q = 0; q < 2; q++) {
            xa[q] = TX ? X[k0 + lk][q * 16 + li] : X[q * 16 + li][k0 + lk];
            yb[q] = Y[k0 + lk][q * 16 + li];
        }
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++) acc[a][b] = mfma16x16x4(xa[a], yb[b], acc[a][b]);
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) O[a * 16 + lk + 4 * r][b * 16 + li] = acc[a][b][r];
    __syncthreads();
}

__global__ __launch_bounds__(64) void k_bj_apply(int np, double *__restrict__ A, double *__restrict__ U,
                                                 PairList pl, const double *__restrict__ Rbuf) {
    __shared__ double T[JG][JG + 1];
    __shared__ double X[JG][JG + 1];
    __shared__ double Ra[JG][JG + 1];
    __shared__ double Rb[JG][JG + 1];
    const int ng = pl.n, lane = threadIdx.x;
    const int t = blockIdx.x;
    if (t < ng * ng) {
        const int a = t / ng, b = t % ng;
        const int Ia = pl.I[a], Ja = pl.J[a], Ib = pl.I[b], Jb = pl.J[b];
        for (int e = lane; e < JG * JG; e += 64) {
            const int r = e / JG, c = e % JG;
            T[r][c] = A[(int64_t)grp_index(r, Ia, Ja) * np + grp_index(c, Ib, Jb)];
            Ra[r][c] = Rbuf[(int64_t)a * JG * JG + e];
            Rb[r][c] = Rbuf[(int64_t)b * JG * JG + e];
        }
        __syncthreads();
        mm32<false>(T, Rb, X);   // X = A_ab R_b
        mm32<true>(Ra, X, T);    // T = R_a^t X
        for (int e = lane; e < JG * JG; e += 64) {
            const int r = e / JG, c = e % JG;
            A[(int64_t)grp_index(r, Ia, Ja) * np + grp_index(c, Ib, Jb)] = T[r][c];
        }
    } else {
        const int u = t - ng * ng;
        const int rt = u / ng, b = u % ng;
        const int Ib = pl.I[b], Jb = pl.J[b];
        for (int e = lane; e < JG * JG; e += 64) {
            const int r = e / JG, c = e % JG;
            T[r][c] = U[(int64_t)(rt * JG + r) * np + grp_index(c, Ib, Jb)];
            Rb[r][c] = Rbuf[(int64_t)b * JG * JG + e];
        }
        __syncthreads();
        mm32<false>(T, Rb, X);   // X = U_rb R_b
        for (int e = lane; e < JG * JG; e += 64) {
            const int r = e / JG, c = e % JG;
            U[(int64_t)(rt * JG + r) * np + grp_index(c, Ib, Jb)] = X[r][c];
        }
    }
}

// A (np x np, zero padded) <- S; U <- I
__global__ void k_bj_init(int n, int np, const double *__restrict__ S, int64_t lds, double *__restrict__ A,
                          double *__restrict__ U) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)np * np) return;
    const int i = (int)(e / np), j = (int)(e % np);
    A[e] = (i < n && j < n) ? S[(int64_t)i * lds + j] : 0.0;
    U[e] = (i == j) ? 1.0 : 0.0;
}

// off-diagonal and total squared Frobenius norms (one workgroup, fixed order)
__global__ __launch_bounds__(1024) void k_bj_norms(int np, const double *__restrict__ A, double *out) {
    __shared__ double so[1024], sd[1024];
    double o = 0.0, d = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)np * np; e += 1024) {
        const double v = A[e];
        if (e / np == e % np) d += v * v;
        else o += v * v;
    }
    so[threadIdx.x] = o;
    sd[threadIdx.x] = d;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            so[threadIdx.x] += so[threadIdx.x + w];
            sd[threadIdx.x] += sd[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = so[0];
        out[1] = sd[0];
    }
}

// G <- 1.5 I - 0.5 G  (one Newton-Schulz step toward (U^t U)^(-1/2))
__global__ void k_newton_schulz(int n, double *G) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    G[e] = ((e / n == e % n) ? 1.5 : 0.0) - 0.5 * G[e];
}

// lam_j = u_j^t (S u_j): column sums of U o (S U), fixed order
__global__ void k_rayleigh_cols(int n, const double *__restrict__ U, int64_t ldu, const double *__restrict__ SU,
                                double *__restrict__ lam) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int i = 0; i < n; i++) s += U[(int64_t)i * ldu + j] * SU[(int64_t)i * n + j];
    lam[j] = s;
}

__global__ void k_copy_mat(int n, const double *__restrict__ a, int64_t lda, double *__restrict__ b, int64_t ldb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    b[(int64_t)(e / n) * ldb + e % n] = a[(int64_t)(e / n) * lda + e % n];
}

// w = lam sorted ascending (ties by index), Uo = columns of X permuted alike
__global__ __launch_bounds__(1024) void k_sort_pairs(int n, const double *__restrict__ lam,
                                                     const double *__restrict__ X, int64_t ldx, double *w,
                                                     double *Uo, int64_t ldo) {
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double wi = lam[i];
        int r = 0;
        for (int j = 0; j < n; j++) r += (lam[j] < wi) || (lam[j] == wi && j < i);
        w[r] = wi;
        for (int k = 0; k < n; k++) Uo[(int64_t)k * ldo + r] = X[(int64_t)k * ldx + i];
    }
}

// eigenvalues ascending (ties by index) and the eigenvector columns alike
__global__ __launch_bounds__(1024) void k_bj_finish(int n, int np, const double *__restrict__ A,
                                                    const double *__restrict__ U, double *w, double *Uo,
                                                    int64_t ldo) {
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double wi = A[(int64_t)i * np + i];
        int r = 0;
        for (int j = 0; j < n; j++) {
            const double wj = A[(int64_t)j * np + j];
            r += (wj < wi) || (wj == wi && j < i);
        }
        w[r] = wi;
        for (int k = 0; k < n; k++) Uo[(int64_t)k * ldo + r] = U[(int64_t)k * np + i];
    }
}

}  // namespace

static int g_syev_sweeps = 0;
int last_syev_sweeps() { return g_syev_sweeps; }

fd_status syev(int n, double *S, int64_t lds, double *w, double *Uo, int64_t ldu, hipStream_t s) {
    if (n < 1 || n > 512) return fail(FD_ERR_INVALID, "syev: need 1 <= n <= 512");
    g_syev_sweeps = 0;
    const int np = (n + JG - 1) / JG * JG;
    const int nbk = np / JB;        // even
    const int ng = nbk / 2;
    const size_t nn = (size_t)np * np;
    double *ws = (double *)workspace((2 * nn + (size_t)ng * JG * JG + 2) * sizeof(double), 1);
    if (!ws) return fail(FD_ERR_OOM, "syev: workspace");
    double *A = ws, *U = ws + nn, *Rbuf = ws + 2 * nn, *nrm = Rbuf + (size_t)ng * JG * JG;
    hipLaunchKernelGGL(k_bj_init, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, n, np, S, lds, A, U);
    FD_HIP(hipGetLastError());
    const double tol = n * 2.220446049250313e-16;
    double prev = INFINITY, rel = 1.0;
    for (int sweep = 0; sweep < 30; sweep++) {
        const double thr2 = std::max(1e-32, 1e-6 * rel * rel);
        for (int rnd = 0; rnd < nbk - 1; rnd++) {
            PairList pl;
            pl.n = ng;
            for (int k = 0; k < ng; k++) {
                auto who = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + rnd) % (nbk - 1); };
                int p = who(k), q = who(nbk - 1 - k);
                pl.I[k] = (unsigned char)std::min(p, q);
                pl.J[k] = (unsigned char)std::max(p, q);
            }
            hipLaunchKernelGGL(k_bj_solve, dim3(ng), dim3(256), 0, s, np, A, pl, Rbuf, thr2, kBjInner);
            FD_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_bj_apply, dim3(2 * ng * ng), dim3(64), 0, s, np, A, U, pl, Rbuf);
            FD_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_bj_norms, dim3(1), dim3(1024), 0, s, np, A, nrm);
        FD_HIP(hipGetLastError());
        double h[2];
        FD_HIP(hipMemcpyAsync(h, nrm, sizeof(h), hipMemcpyDeviceToHost, s));
        FD_HIP(hipStreamSynchronize(s));
        const double off = std::sqrt(h[0]), fro = std::sqrt(h[0] + h[1]);
        g_syev_sweeps = sweep + 1;
        if (!std::isfinite(off)) return fail(FD_ERR_BREAKDOWN, "syev: non-finite matrix");
        // converged, or stalled at the rounding floor of the tile updates
        if (off <= tol * fro || (off > 0.9 * prev && off <= 10 * tol * fro)) break;
        prev = off;
        rel = off / fro;
    }
    hipLaunchKernelGGL(k_bj_finish, dim3(1), dim3(1024), 0, s, n, np, A, U, w, Uo, ldu);
    FD_HIP(hipGetLastError());
    // The product of many block rotations drifts from orthogonality by a few
    // hundred ulps; one Newton-Schulz step U <- U (3 I - U^t U) / 2 squares
    // that error.  A is free now and holds the n x n Gram matrix.
    FD_TRY(gram(n, n, n, Uo, ldu, Uo, ldu, A, n, true, s));
    hipLaunchKernelGGL(k_newton_schulz, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, n, A);
    FD_HIP(hipGetLastError());
    FD_TRY(rotate(n, n, n, Uo, ldu, A, n, s));
    // Eigenvalues as Rayleigh quotients u_j^t S u_j of the untouched input:
    // error O(eps ||S||) plus the square of the eigenvector error, instead of
    // the rounding the tile updates left on the diagonal of A.
    const unsigned gb = (unsigned)((n * n + 255) / 256);
    hipLaunchKernelGGL(k_copy_mat, dim3(gb), dim3(256), 0, s, n, S, lds, U, (int64_t)n);
    FD_HIP(hipGetLastError());
    FD_TRY(rotate(n, n, n, U, n, Uo, ldu, s));  // U <- S Uo
    hipLaunchKernelGGL(k_rayleigh_cols, dim3((n + 255) / 256), dim3(256), 0, s, n, Uo, ldu, U, A);
    FD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_copy_mat, dim3(gb), dim3(256), 0, s, n, Uo, ldu, U, (int64_t)n);
    FD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sort_pairs, dim3(1), dim3(1024), 0, s, n, A, U, (int64_t)n, w, Uo, ldu);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

// ------------------------------------------------------ SVQB / CholQR ----
namespace {

// G (n x n, ld n) -> Dg G Dg in place; d[i] = 1/sqrt(G_ii) (1 for G_ii <= 0)
__global__ void k_scale_gram(int n, double *G, double *d) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double g = G[i * n + i];
        d[i] = (g > 0.0) ? 1.0 / sqrt(g) : 1.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) G[e] *= d[e / n] * d[e % n];
}

// Q = Dg U L^-1/2 with L clipped at 1e-14 max(L); keep[j] = L_j > floor;
// *rank = -1 when an eigenvalue is not finite
__global__ void k_svqb_q(int n, const double *d, const double *lam, const double *U, double *Q,
                         int *keep, int *rank) {
    __shared__ double fl;
    __shared__ int cnt;
    __shared__ int finite;
    if (threadIdx.x == 0) {
        double mx = 0.0;
        int f = 1;
        for (int j = 0; j < n; j++) {
            mx = fmax(mx, lam[j]);
            f &= isfinite(lam[j]) ? 1 : 0;
        }
        fl = 1e-14 * mx;
        cnt = 0;
        finite = f;
    }
    __syncthreads();
    if (!finite) {  // a non-finite Gram matrix: rank -1, nothing kept
        for (int j = threadIdx.x; j < n; j += blockDim.x) keep[j] = 0;
        if (threadIdx.x == 0) *rank = -1;
        return;
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const bool k = lam[j] > fl && fl > 0.0;
        keep[j] = k ? 1 : 0;
        if (k) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        const double l = fmax(lam[j], fl > 0.0 ? fl : 1.0);
        Q[e] = d[i] * U[e] / sqrt(l);
    }
    if (threadIdx.x == 0) *rank = cnt;
}

// G = R^t R (R upper), then Q = R^-1; ok = 0 if a pivot is not positive
// Cholesky G = R^t R (upper R in place) and Q = R^-1.  *ok = 0 when a pivot
// falls to 1e-14 n of the matrix's own diagonal entry or below (the block is
// numerically rank deficient: its Gram matrix carries no information in
// that direction, and CholQR would return a non-orthonormal block), or, with
// near_identity set (the second pass of CholQR2), when some entry of G is
// more than 0.5 away from the identity (the first pass has already failed).
__global__ __launch_bounds__(1024) void k_cholinv(int n, double *G, double *Q, int *ok, int near_identity) {
    __shared__ int good;
    __shared__ double d0[512];
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
            if (threadIdx.x == 0) *ok = 0;
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
            const int i = k + 1 + e / rem, j = k + 1 + e % rem;
            if (j >= i) G[i * n + j] -= G[k * n + i] * G[k * n + j];
        }
        __syncthreads();
    }
    __syncthreads();
    if (!good) {
        if (threadIdx.x == 0) *ok = 0;
        return;
    }
    // column j of X = R^-1: back substitution, one column per thread
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        for (int i = n - 1; i >= 0; i--) {
            double s = (i == j) ? 1.0 : 0.0;
            if (i > j) {
                Q[i * n + j] = 0.0;
                continue;
            }
            for (int k = i + 1; k <= j; k++) s -= G[i * n + k] * Q[k * n + j];
            Q[i * n + j] = s / G[i * n + i];
        }
    }
    if (threadIdx.x == 0) *ok = 1;
}

// The same for n <= 128 with G held in LDS (stride n + 1): one barrier per
// elimination step and per column of the inverse.  Step k updates the
// trailing rows with the unscaled row k (g_ij -= g_ki g_kj / g_kk) and scales
// row k one step later, when no thread reads it any more.  X = R^-1 is built
// column by column (x_jj = 1 / r_jj, x_ij = -x_jj sum_{i <= k < j} x_ik r_kj)
// into the lower triangle (x_ij at [j][i]), eight threads per dot product.
constexpr int kCholLds = 128;
__global__ __launch_bounds__(1024) void k_cholinv_lds(int n, const double *__restrict__ G, double *__restrict__ Q,
                                                      int *ok, int near_identity) {
    __shared__ double L[kCholLds * (kCholLds + 1)];
    __shared__ double d0[kCholLds], dinv[kCholLds];
    __shared__ int good;
    const int tid = threadIdx.x, ld = n + 1;
    if (tid == 0) good = 1;
    for (int e = tid; e < n * n; e += 1024) {
        const int i = e / n, j = e % n;
        const double g = G[e];
        L[i * ld + j] = g;
        if (i == j) d0[i] = g;
        if (near_identity && !(fabs(g - (i == j ? 1.0 : 0.0)) <= 0.5)) good = 0;
    }
    __syncthreads();
    const double rel = 1e-14 * (double)n;
    double rprev = 1.0;  // r_{k-1,k-1}
    for (int k = 0; k < n && good; k++) {
        const double piv = L[k * ld + k];
        const bool pass = piv > rel * d0[k];
        // scale row k - 1 right of the diagonal; no thread reads it now
        if (k > 0)
            for (int j = k + tid; j < n; j += 1024) L[(k - 1) * ld + j] /= rprev;
        if (!pass) {
            good = 0;  // every thread read the same pivot
            break;
        }
        const double inv = 1.0 / piv;
        // trailing upper triangle, threads as 32 x 32 (row step 32, column step 32)
        for (int i = k + 1 + (tid >> 5); i < n; i += 32) {
            const double f = L[k * ld + i] * inv;
            for (int j = i + ((tid - i) & 31); j < n; j += 32) L[i * ld + j] -= f * L[k * ld + j];
        }
        rprev = sqrt(piv);
        __syncthreads();
        if (tid == 0) L[k * ld + k] = rprev;
    }
    __syncthreads();
    if (!good) {
        if (tid == 0) *ok = 0;
        return;
    }
    // row n - 1 has nothing right of its diagonal: every row is scaled
    for (int i = tid; i < n; i += 1024) dinv[i] = 1.0 / L[i * ld + i];
    __syncthreads();
    const int i = tid >> 3, t = tid & 7;
    for (int j = 1; j < n; j++) {
        double acc = 0.0;
        if (i < j) {
            for (int k = i + t; k < j; k += 8) {
                const double xik = (k == i) ? dinv[i] : L[k * ld + i];
                acc += xik * L[k * ld + j];
            }
        }
        acc += __shfl_xor(acc, 1, 8);
        acc += __shfl_xor(acc, 2, 8);
        acc += __shfl_xor(acc, 4, 8);
        if (i < j && t == 0) L[j * ld + i] = -dinv[j] * acc;
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += 1024) {
        const int r = e / n, c = e % n;
        Q[e] = c > r ? L[c * ld + r] : (c == r ? dinv[r] : 0.0);
    }
    if (tid == 0) *ok = 1;
}

__global__ void k_minus_identity(int n, const double *__restrict__ G, double *__restrict__ E) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n * n) E[e] = G[e] - ((e / n == e % n) ? 1.0 : 0.0);
}

// Second orthogonalization pass (the Gram matrix G = I + E of a block that
// one pass has already orthonormalized to about kappa eps): Q = G^-1/2 by its
// series I - E/2 + 3 E^2/8 (omitted terms below 0.32 |E|^3), with E2 = E^2
// given.  *ok = 0 (Q untouched) when n max|E_ij| > 1e-5, which bounds |E|_2.
__global__ __launch_bounds__(1024) void k_lowdin(int n, const double *__restrict__ G, const double *__restrict__ E2,
                                                 double *__restrict__ Q, int *ok) {
    __shared__ int good;
    if (threadIdx.x == 0) good = 1;
    __syncthreads();
    const double lim = 1e-5 / (double)n;
    for (int e = threadIdx.x; e < n * n; e += 1024) {
        const double d = G[e] - ((e / n == e % n) ? 1.0 : 0.0);
        if (!(fabs(d) <= lim)) good = 0;
    }
    __syncthreads();
    if (!good) {
        if (threadIdx.x == 0) *ok = 0;
        return;
    }
    for (int e = threadIdx.x; e < n * n; e += 1024) {
        const double d = G[e] - ((e / n == e % n) ? 1.0 : 0.0);
        Q[e] = ((e / n == e % n) ? 1.0 : 0.0) - 0.5 * d + 0.375 * E2[e];
    }
    if (threadIdx.x == 0) *ok = 1;
}

}  // namespace

fd_status svqb_transform(int n, double *G, double *Q, double *work, int *keep, int *rank_dev,
                         hipStream_t s) {
    // work: d (n) + lam (n) + U (n*n)
    double *d = work, *lam = work + n, *U = work + 2 * n;
    hipLaunchKernelGGL(k_scale_gram, dim3(1), dim3(1024), 0, s, n, G, d);
    FD_HIP(hipGetLastError());
    FD_TRY(syev(n, G, n, lam, U, n, s));
    hipLaunchKernelGGL(k_svqb_q, dim3(1), dim3(1024), 0, s, n, d, lam, U, Q, keep, rank_dev);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status cholqr_transform(int n, double *G, double *Q, int *ok_dev, bool second_pass, hipStream_t s) {
    if (n > 512) return fail(FD_ERR_INVALID, "CholQR: n > 512");
    if (n <= kCholLds)
        hipLaunchKernelGGL(k_cholinv_lds, dim3(1), dim3(1024), 0, s, n, G, Q, ok_dev, second_pass ? 1 : 0);
    else
        hipLaunchKernelGGL(k_cholinv, dim3(1), dim3(1024), 0, s, n, G, Q, ok_dev, second_pass ? 1 : 0);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status lowdin_transform(int n, const double *G, double *E, double *E2, double *Q, int *ok_dev, hipStream_t s) {
    // E = G - I, E2 = E^t E = E^2 (E is symmetric)
    hipLaunchKernelGGL(k_minus_identity, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, n, G, E);
    FD_HIP(hipGetLastError());
    FD_TRY(gram(n, n, n, E, n, E, n, E2, n, true, s));
    hipLaunchKernelGGL(k_lowdin, dim3(1), dim3(1024), 0, s, n, G, E2, Q, ok_dev);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

// ----------------------------------------------------- residual norms ----
namespace {

__global__ __launch_bounds__(256) void k_resid_part(int64_t D, int n, const double *__restrict__ V,
                                                    const double *__restrict__ W, int64_t ld,
                                                    const double *__restrict__ theta, int64_t rpb,
                                                    double *__restrict__ P) {
    const int64_t r0 = (int64_t)blockIdx.x * rpb, r1 = min(D, r0 + rpb);
    for (int j = threadIdx.x; j < n; j += 256) {
        const double th = theta[j];
        double s = 0.0;
        for (int64_t r = r0; r < r1; r++) {
            const double e = W[r * ld + j] - th * V[r * ld + j];
            s += e * e;
        }
        P[(int64_t)blockIdx.x * n + j] = s;
    }
}

__global__ void k_resid_final(int nblk, int n, const double *P, double *rho) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int b = 0; b < nblk; b++) s += P[(int64_t)b * n + j];
    rho[j] = sqrt(s);
}

}  // namespace

fd_status col_resid(int64_t D, int n, const double *V, const double *W, int64_t ld, const double *theta,
                    double *rho, hipStream_t s) {
    int64_t rpb = std::max<int64_t>(64, (D + 2047) / 2048);
    int nblk = (int)((D + rpb - 1) / rpb);
    double *P = (double *)workspace((size_t)nblk * n * sizeof(double), 2);
    if (!P) return fail(FD_ERR_OOM, "resid: workspace");
    hipLaunchKernelGGL(k_resid_part, dim3(nblk), dim3(256), 0, s, D, n, V, W, ld, theta, rpb, P);
    FD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_resid_final, dim3((n + 255) / 256), dim3(256), 0, s, nblk, n, P, rho);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

// ------------------------------------------------------ column dots ----
namespace {
__global__ __launch_bounds__(256) void k_coldot_part(int64_t D, int n, const double *__restrict__ A, int64_t lda,
                                                     const double *__restrict__ B, int64_t ldb, int64_t rpb,
                                                     double *__restrict__ P) {
    const int64_t r0 = (int64_t)blockIdx.x * rpb, r1 = min(D, r0 + rpb);
    for (int j = threadIdx.x; j < n; j += 256) {
        double s = 0.0;
        for (int64_t r = r0; r < r1; r++) s += A[r * lda + j] * B[r * ldb + j];
        P[(int64_t)blockIdx.x * n + j] = s;
    }
}

__global__ void k_coldot_final(int nblk, int n, const double *P, double *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int b = 0; b < nblk; b++) s += P[(int64_t)b * n + j];
    out[j] = s;
}

__global__ void k_copy_block(int64_t D, int n, const double *__restrict__ a, int64_t la, double *__restrict__ b,
                             int64_t lb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D * n) return;
    const int64_t i = e / n;
    const int j = (int)(e % n);
    b[i * lb + j] = a[i * la + j];
}
}  // namespace

fd_status col_dots(int64_t D, int n, const double *A, int64_t lda, const double *B, int64_t ldb, double *out,
                   hipStream_t s, double *P) {
    int64_t rpb = std::max<int64_t>(64, (D + 2047) / 2048);
    int nblk = (int)((D + rpb - 1) / rpb);
    if (!P) P = (double *)workspace((size_t)nblk * n * sizeof(double), 2);
    if (!P) return fail(FD_ERR_OOM, "col_dots: workspace");
    hipLaunchKernelGGL(k_coldot_part, dim3(nblk), dim3(256), 0, s, D, n, A, lda, B, ldb, rpb, P);
    FD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_coldot_final, dim3((n + 255) / 256), dim3(256), 0, s, nblk, n, P, out);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status copy_block(int64_t D, int n, const double *src, int64_t lds, double *dst, int64_t ldd, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_block, dim3((unsigned)((D * n + 255) / 256)), dim3(256), 0, s, D, n, src, lds, dst, ldd);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

// ------------------------------------------------ static device scratch ----
// A fixed array for the entry points that must not allocate (each device
// the library runs on holds its own copy until the process ends).  Host code
// never names the array in a kernel argument or a copy: its address on the
// current device comes from hipGetSymbolAddress, resolved once per device.
namespace {
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};
}  // namespace

fd_status scratch_ptr(void **out) {
    int dev = 0;
    FD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(FD_ERR_UNSUPPORTED, "scratch: device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch: symbol address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FD_OK;
}

// ------------------------------------------------------------- Lanczos ----
// Vectors of the Lanczos basis are stored one after another (vector t at
// Q + t * D, each contiguous), so the SpMV on one of them and the
// projections below read whole rows of memory.
namespace {
// P[t * nblk + b] = sum over rows of block b of Q_t[i] w[i], t = blockIdx.y
__global__ __launch_bounds__(256) void k_lz_proj(int64_t D, const double *__restrict__ Q,
                                                 const double *__restrict__ w, int64_t rpb, double *__restrict__ P) {
    const int t = blockIdx.y;
    const double *q = Q + (int64_t)t * D;
    const int64_t r0 = (int64_t)blockIdx.x * rpb, r1 = min(D, r0 + rpb);
    double acc = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) acc += q[r] * w[r];
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) P[(int64_t)t * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_lz_final(int nblk, int n, const double *__restrict__ P, double *__restrict__ c) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; b++) acc += P[(int64_t)t * nblk + b];
    c[t] = acc;
}

// w[i] -= sum_t Q_t[i] c[t]
__global__ __launch_bounds__(256) void k_lz_sub(int64_t D, int n, const double *__restrict__ Q,
                                                const double *__restrict__ c, double *__restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= D) return;
    double acc = 0.0;
    for (int t = 0; t < n; t++) acc = fma(Q[(int64_t)t * D + i], c[t], acc);
    w[i] -= acc;
}

__global__ __launch_bounds__(256) void k_lz_scale(int64_t D, double *__restrict__ w, double f) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < D) w[i] *= f;
}

// u_i = 2 U_i - 1, U_i the i-th output (from 0) of SplitMix64(seed)
__device__ __forceinline__ uint64_t lz_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__global__ __launch_bounds__(256) void k_lz_start(int64_t D, double *__restrict__ q, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= D) return;
    const uint64_t z = lz_mix(seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL);
    q[i] = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}
}  // namespace

fd_status lz_dots(int64_t D, int n, const double *Q, const double *w, double *c, double *P, int nblk,
                  hipStream_t s) {
    const int64_t rpb = (D + nblk - 1) / nblk;
    hipLaunchKernelGGL(k_lz_proj, dim3((unsigned)nblk, (unsigned)n), dim3(256), 0, s, D, Q, w, rpb, P);
    FD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_lz_final, dim3((n + 63) / 64), dim3(64), 0, s, nblk, n, P, c);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status lz_sub(int64_t D, int n, const double *Q, const double *c, double *w, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_sub, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, D, n, Q, c, w);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status lz_scale(int64_t D, double *w, double f, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_scale, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, D, w, f);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status lz_start(int64_t D, double *q, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_start, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, D, q, seed);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

// ------------------------------------------------ strided block copy ----
namespace {
// rows of `w` units of U (4, 8 or 16 bytes): b[i * lb + j] = a[i * la + j]
template <typename U>
__global__ __launch_bounds__(256) void k_copy2d(int64_t D, int w, const U *__restrict__ a, int64_t la,
                                                U *__restrict__ b, int64_t lb) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= D * w) return;
    const int64_t i = e / w;
    const int j = (int)(e % w);
    __builtin_nontemporal_store(__builtin_nontemporal_load(a + i * la + j), b + i * lb + j);
}
}  // namespace

fd_status copy_rows(int64_t D, int64_t row_bytes, const void *src, int64_t src_ld_bytes, void *dst,
                    int64_t dst_ld_bytes, hipStream_t s) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const uintptr_t al = (uintptr_t)src | (uintptr_t)dst | (uintptr_t)row_bytes | (uintptr_t)src_ld_bytes |
                         (uintptr_t)dst_ld_bytes;
    const int64_t u = (al % 16 == 0) ? 16 : (al % 8 == 0) ? 8 : 4;
    if (al % 4) return fail(FD_ERR_INVALID, "copy_rows: 4-byte alignment needed");
    const int w = (int)(row_bytes / u);
    const unsigned g = (unsigned)((D * w + 255) / 256);
    if (u == 16)
        hipLaunchKernelGGL(k_copy2d<f4>, dim3(g), dim3(256), 0, s, D, w, (const f4 *)src, src_ld_bytes / 16,
                           (f4 *)dst, dst_ld_bytes / 16);
    else if (u == 8)
        hipLaunchKernelGGL(k_copy2d<double>, dim3(g), dim3(256), 0, s, D, w, (const double *)src, src_ld_bytes / 8,
                           (double *)dst, dst_ld_bytes / 8);
    else
        hipLaunchKernelGGL(k_copy2d<float>, dim3(g), dim3(256), 0, s, D, w, (const float *)src, src_ld_bytes / 4,
                           (float *)dst, dst_ld_bytes / 4);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

// --------------------------------------------------- element-wise kernels --
namespace {

__device__ __forceinline__ uint64_t smix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// N(0,1) for entry (i, j) of a D x n block: SplitMix64 outputs number
// 2 (i n + j) + 1 and + 2 of the stream `seed` (counter based), Box-Muller
// with u1 -> 1 - u1 so that the logarithm stays finite.
__device__ __forceinline__ double normal_at(uint64_t seed, int64_t i, int n, int j) {
    const uint64_t c = 2 * ((uint64_t)i * (uint64_t)n + (uint64_t)j);
    const uint64_t g = 0x9E3779B97F4A7C15ULL;
    const double u1 = (double)(smix(seed + (c + 1) * g) >> 11) * 0x1.0p-53;
    const double u2 = (double)(smix(seed + (c + 2) * g) >> 11) * 0x1.0p-53;
    return sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
}

__global__ void k_fill_normal(int64_t D, int n, double *V, int64_t ldv, const int *keep, uint64_t seed) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D * n) return;
    const int64_t i = e / n;
    const int j = (int)(e % n);
    if (keep && keep[j]) return;
    V[i * ldv + j] = normal_at(seed, i, n, j);
}

__global__ void k_f64_to_f32(int64_t D, int n, const double *a, int64_t la, float *b, int64_t lb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D * n) return;
    const int64_t i = e / n;
    const int j = (int)(e % n);
    b[i * lb + j] = (float)a[i * la + j];
}

__global__ void k_f32_to_f64(int64_t D, int n, const float *a, int64_t la, double *b, int64_t lb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D * n) return;
    const int64_t i = e / n;
    const int j = (int)(e % n);
    b[i * lb + j] = (double)a[i * la + j];
}

__global__ void k_gather_cols(int64_t D, int n, const double *a, int64_t la, const int *idx, double *b,
                              int64_t lb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D * n) return;
    const int64_t i = e / n;
    const int j = (int)(e % n);
    b[i * lb + j] = a[i * la + idx[j]];
}

__global__ void k_symmetrize(int n, double *H) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int i = e / n, j = e % n;
    if (i < j) {
        const double a = 0.5 * (H[i * n + j] + H[j * n + i]);
        H[i * n + j] = a;
        H[j * n + i] = a;
    }
}

unsigned nblocks(int64_t tot) { return (unsigned)((tot + 255) / 256); }

// STREAM-style kernels (the paper measures b_m with STREAM): 16-byte
// non-temporal loads and stores, four per thread in flight, grid-stride over
// n/2 pairs of doubles (a probe of copy variants on MI355X found this shape
// fastest).
typedef double d2v __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void k_stream(int op, int64_t n2, const d2v *__restrict__ a,
                                                const d2v *__restrict__ b, d2v *__restrict__ c, double sc) {
    const int64_t stride = (int64_t)gridDim.x * 256 * 4;
    int64_t i = (int64_t)blockIdx.x * 256 * 4 + threadIdx.x;
    d2v acc = (d2v)0;
    for (; i + 3 * 256 < n2; i += stride) {
        d2v r[4];
        if (op == 3) {
#pragma unroll
            for (int u = 0; u < 4; u++) __builtin_nontemporal_store((d2v)sc, c + i + u * 256);
            continue;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) r[u] = __builtin_nontemporal_load(a + i + u * 256);
        if (op == 2) {
#pragma unroll
            for (int u = 0; u < 4; u++) acc += r[u];
            continue;
        }
        if (op == 1) {
#pragma unroll
            for (int u = 0; u < 4; u++) r[u] += sc * __builtin_nontemporal_load(b + i + u * 256);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) __builtin_nontemporal_store(r[u], c + i + u * 256);
    }
    for (; i < n2; i += 256) {  // tail: the remaining elements of this block's last tile
        if (op == 3) {
            __builtin_nontemporal_store((d2v)sc, c + i);
            continue;
        }
        d2v r = __builtin_nontemporal_load(a + i);
        if (op == 2) {
            acc += r;
            continue;
        }
        if (op == 1) r += sc * __builtin_nontemporal_load(b + i);
        __builtin_nontemporal_store(r, c + i);
    }
    // read-only pass: one partial sum per thread, so that the loads stay live
    if (op == 2) c[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

}  // namespace

fd_status stream_op(int op, int64_t n, const double *a, const double *b, double *c, double sc, hipStream_t s) {
    if (n < 2 || (n & 1) || op < 0 || op > 3 || !c || (op != 3 && !a) || (op == 1 && !b) ||
        ((uintptr_t)a | (uintptr_t)c | (uintptr_t)b) % 16)
        return fail(FD_ERR_INVALID, "stream: need even n, 16-byte aligned arrays, op 0..3");
    const int64_t n2 = n / 2;
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>((n2 + 1023) / 1024, 16384));
    // the read-only pass writes one partial sum (16 bytes) per thread into c
    if (op == 2 && g * 256 > n2) return fail(FD_ERR_INVALID, "stream: read-only pass needs n >= 2^19");
    hipLaunchKernelGGL(k_stream, dim3((unsigned)g), dim3(256), 0, s, op, n2, (const d2v *)a, (const d2v *)b,
                       (d2v *)c, sc);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status fill_normal(int64_t D, int n, double *V, int64_t ldv, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_normal, dim3(nblocks(D * n)), dim3(256), 0, s, D, n, V, ldv, (const int *)nullptr,
                       seed);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status refill_random(int64_t D, int n, double *V, int64_t ldv, const int *keep, uint64_t seed,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_fill_normal, dim3(nblocks(D * n)), dim3(256), 0, s, D, n, V, ldv, keep, seed);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status convert_f64_f32(int64_t D, int n, const double *src, int64_t lds, float *dst, int64_t ldd,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(nblocks(D * n)), dim3(256), 0, s, D, n, src, lds, dst, ldd);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status convert_f32_f64(int64_t D, int n, const float *src, int64_t lds, double *dst, int64_t ldd,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_f32_to_f64, dim3(nblocks(D * n)), dim3(256), 0, s, D, n, src, lds, dst, ldd);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status gather_cols(int64_t D, int n, const double *src, int64_t lds, const int *idx, double *dst,
                      int64_t ldd, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_cols, dim3(nblocks(D * n)), dim3(256), 0, s, D, n, src, lds, idx, dst, ldd);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

fd_status symmetrize(int n, double *H, hipStream_t s) {
    hipLaunchKernelGGL(k_symmetrize, dim3(nblocks((int64_t)n * n)), dim3(256), 0, s, n, H);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

namespace {
// Lehmann pencil from G2 = W^t W, G1 = V^t W, G0 = V^t V (W = A V):
// B = ((A - rho) V)^t ((A - rho) V) = G2 - rho (G1 + G1^t) + rho^2 G0 and
// S = V^t (A - rho) V = (G1 + G1^t) / 2 - rho G0.
__global__ void k_lehmann_prep(int n, const double *G2, const double *G1, const double *G0, double rho, double *B,
                               double *S) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int i = e / n, j = e % n;
    const double g1 = G1[i * n + j] + G1[j * n + i];
    B[e] = G2[e] - rho * g1 + rho * rho * G0[e];
    S[e] = 0.5 * g1 - rho * G0[e];
}
}  // namespace

fd_status lehmann_pencil(int n, const double *G2, const double *G1, const double *G0, double rho, double *B,
                         double *S, hipStream_t s) {
    hipLaunchKernelGGL(k_lehmann_prep, dim3(nblocks((int64_t)n * n)), dim3(256), 0, s, n, G2, G1, G0, rho, B, S);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

}  // namespace fd
