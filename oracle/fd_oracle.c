/*
 * fd_oracle.c -- plain FP64 CPU oracle for the filter-diagonalization hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test suite, the package smoke check and the CPU
 * baseline leg of the benchmark load it (through ctypes, see oracle.py).  It
 * shares no source with the HIP path.
 *
 * Everything here is the plain definition written out, in FP64, with loops a
 * reader can check against the paper by eye:
 *   - generated Hamiltonians (Hubbard ring, 3D Anderson lattice, diagonal)
 *     as canonical CSR (columns ascending, diagonal always stored);
 *   - the SELL-C-sigma layout of such a CSR matrix;
 *   - block SpMV  y_i = sum_j A_ij x_j  on row-major blocks of nb vectors
 *     (Sec. 3.1, Eq. SpMVprocess; row-major vector storage as Sec. 3.1 asks);
 *   - the polynomial filter V -> p[A] V = sum_k mu_k T_k(alpha A + beta) V,
 *     evaluated with the Chebyshev three-term recurrence, one unfused BLAS-1
 *     pass at a time (Sec. 2, Alg. 2 caption: n >= 2, n SpMVs, workspaces
 *     W1, W2, scaling alpha, beta from the inclusion interval);
 *   - the Chebyshev expansion coefficients of a window function with Jackson
 *     damping (Sec. 2 defers the window to its references; the reading used
 *     is the indicator of the target interval, damped with the Jackson kernel);
 *   - the SplitMix64 generator (Steele, Lea, Flood, OOPSLA 2014) that draws the
 *     Anderson disorder from a seed.
 *
 * Parity pins for every function are in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads the OpenMP loops of this file use */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* SplitMix64: state advances by the golden gamma, output is the mix of the
 * new state (Steele, Lea & Flood 2014).  u = top 53 bits * 2^-53 in [0,1).  */
uint64_t orc_splitmix64(uint64_t *state)
{
    uint64_t z;
    *state = *state + 0x9E3779B97F4A7C15ULL;
    z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double orc_uniform(uint64_t *state)
{
    return (double)(orc_splitmix64(state) >> 11) * (1.0 / 9007199254740992.0);
}

void orc_uniform_fill(uint64_t seed, int64_t n, double *out)
{
    uint64_t s = seed;
    for (int64_t i = 0; i < n; i++) out[i] = orc_uniform(&s);
}

/* ------------------------------------------------------------------------ */
/* binomial coefficient by Pascal's rule (exact for the sizes used here)    */
int64_t orc_binom(int n, int k)
{
    if (k < 0 || k > n) return 0;
    int64_t c = 1;
    for (int i = 1; i <= k; i++) c = c * (n - k + i) / i;
    return c;
}

static int popcount64(uint64_t x)
{
    int c = 0;
    while (x) { c += (int)(x & 1u); x >>= 1; }
    return c;
}

/* All L-bit masks with exactly N bits set, in increasing integer order. */
static int64_t enumerate_masks(int L, int N, uint64_t *out)
{
    int64_t cnt = 0;
    for (uint64_t m = 0; m < (1ULL << L); m++)
        if (popcount64(m) == N) {
            if (out) out[cnt] = m;
            cnt++;
        }
    return cnt;
}

/* position of mask m in the sorted list (plain binary search) */
static int64_t mask_rank(const uint64_t *list, int64_t n, uint64_t m)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (list[mid] == m) return mid;
        if (list[mid] < m) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* One species: all states reachable from mask m by one nearest-neighbour hop
 * on the ring (or open chain).  Fermion sign from Jordan-Wigner ordering of
 * the sites 0..L-1 of that species: a hop across bond (i, j) picks up
 * (-1)^(number of occupied sites strictly between i and j).  For an inner
 * bond that number is 0; for the wrap bond (L-1, 0) it is N-1.
 * Writes (new mask, matrix element) pairs; returns how many.               */
static int hops(int L, int periodic, double t, uint64_t m,
                uint64_t *nm, double *el)
{
    int c = 0;
    int nbonds = periodic ? L : L - 1;
    for (int b = 0; b < nbonds; b++) {
        int i = b, j = (b + 1) % L;
        int oi = (int)((m >> i) & 1u), oj = (int)((m >> j) & 1u);
        if (oi == oj) continue;
        uint64_t m2 = m ^ (1ULL << i) ^ (1ULL << j);
        int lo = i < j ? i : j, hi = i < j ? j : i;
        int between = 0;
        for (int s = lo + 1; s < hi; s++) between += (int)((m >> s) & 1u);
        double sign = (between % 2 == 0) ? 1.0 : -1.0;
        nm[c] = m2;
        el[c] = -t * sign;
        c++;
    }
    return c;
}

/* Hubbard ring: H = -t sum_<ij>,s (c+_is c_js + h.c.) + U sum_i n_iu n_id.
 * Row index = rank(up mask) * C(L, n_dn) + rank(down mask).  The diagonal
 * U * popcount(up & down) is always stored.  Returns D and nnz.          */
int orc_hubbard_size(int L, int nup, int ndn, int periodic, double t,
                     int64_t *D, int64_t *nnz)
{
    if (L < 3 || L > 30 || nup < 0 || nup > L || ndn < 0 || ndn > L) return 1;
    int64_t nu = orc_binom(L, nup), nd = orc_binom(L, ndn);
    uint64_t *mu = malloc(sizeof(uint64_t) * nu), *md = malloc(sizeof(uint64_t) * nd);
    enumerate_masks(L, nup, mu);
    enumerate_masks(L, ndn, md);
    uint64_t tmpm[64];
    double tmpe[64];
    int64_t cu = 0, cd = 0;
    for (int64_t a = 0; a < nu; a++) cu += hops(L, periodic, t, mu[a], tmpm, tmpe);
    for (int64_t a = 0; a < nd; a++) cd += hops(L, periodic, t, md[a], tmpm, tmpe);
    *D = nu * nd;
    /* t == 0 stores no hopping entries (exact zeros are never stored)     */
    *nnz = nu * nd + (t != 0.0 ? (cu * nd + cd * nu) : 0);
    free(mu);
    free(md);
    return 0;
}

int orc_hubbard_csr(int L, int nup, int ndn, int periodic, double t, double U,
                    int64_t *rowptr, uint32_t *col, double *val)
{
    if (L < 3 || L > 30) return 1;
    int64_t nu = orc_binom(L, nup), nd = orc_binom(L, ndn);
    uint64_t *mu = malloc(sizeof(uint64_t) * nu), *md = malloc(sizeof(uint64_t) * nd);
    enumerate_masks(L, nup, mu);
    enumerate_masks(L, ndn, md);
    int64_t k = 0;
    rowptr[0] = 0;
    for (int64_t a = 0; a < nu; a++) {
        for (int64_t b = 0; b < nd; b++) {
            int64_t row = a * nd + b;
            /* collect the row's entries, then sort by column (insertion) */
            int64_t cols[128];
            double vals[128];
            int n = 0;
            cols[n] = row;
            vals[n] = U * (double)popcount64(mu[a] & md[b]);
            n++;
            uint64_t nm[64];
            double el[64];
            if (t != 0.0) {
                int h = hops(L, periodic, t, mu[a], nm, el);
                for (int q = 0; q < h; q++) {
                    cols[n] = mask_rank(mu, nu, nm[q]) * nd + b;
                    vals[n] = el[q];
                    n++;
                }
                h = hops(L, periodic, t, md[b], nm, el);
                for (int q = 0; q < h; q++) {
                    cols[n] = a * nd + mask_rank(md, nd, nm[q]);
                    vals[n] = el[q];
                    n++;
                }
            }
            for (int p = 1; p < n; p++) {
                int64_t c = cols[p];
                double v = vals[p];
                int q = p - 1;
                while (q >= 0 && cols[q] > c) {
                    cols[q + 1] = cols[q];
                    vals[q + 1] = vals[q];
                    q--;
                }
                cols[q + 1] = c;
                vals[q + 1] = v;
            }
            for (int p = 0; p < n; p++) {
                col[k] = (uint32_t)cols[p];
                val[k] = vals[p];
                k++;
            }
            rowptr[row + 1] = k;
        }
    }
    free(mu);
    free(md);
    return 0;
}

/* 3D Anderson lattice, L^3 sites, site (x,y,z) -> i = x + L y + L^2 z,
 * periodic nearest-neighbour hopping -t, on-site energy W (u - 1/2) with u
 * drawn from SplitMix64(seed) in row order after the first `skip` draws.  */
int orc_anderson_csr(int L, double t, double W, uint64_t seed, int64_t skip,
                     int64_t *rowptr, uint32_t *col, double *val)
{
    if (L < 3 || skip < 0) return 1;
    int64_t D = (int64_t)L * L * L;
    uint64_t s = seed;
    for (int64_t k = 0; k < skip; k++) (void)orc_uniform(&s);
    int64_t k = 0;
    rowptr[0] = 0;
    for (int64_t i = 0; i < D; i++) {
        int64_t x = i % L, y = (i / L) % L, z = i / ((int64_t)L * L);
        int64_t cols[7];
        double vals[7];
        double eps = W * (orc_uniform(&s) - 0.5);
        cols[0] = i;                                   vals[0] = eps;
        cols[1] = ((x + 1) % L) + L * y + (int64_t)L * L * z;       vals[1] = -t;
        cols[2] = ((x + L - 1) % L) + L * y + (int64_t)L * L * z;   vals[2] = -t;
        cols[3] = x + L * ((y + 1) % L) + (int64_t)L * L * z;       vals[3] = -t;
        cols[4] = x + L * ((y + L - 1) % L) + (int64_t)L * L * z;   vals[4] = -t;
        cols[5] = x + L * y + (int64_t)L * L * ((z + 1) % L);       vals[5] = -t;
        cols[6] = x + L * y + (int64_t)L * L * ((z + L - 1) % L);   vals[6] = -t;
        for (int p = 1; p < 7; p++) {
            int64_t c = cols[p];
            double v = vals[p];
            int q = p - 1;
            while (q >= 0 && cols[q] > c) {
                cols[q + 1] = cols[q];
                vals[q + 1] = vals[q];
                q--;
            }
            cols[q + 1] = c;
            vals[q + 1] = v;
        }
        for (int p = 0; p < 7; p++) {
            col[k] = (uint32_t)cols[p];
            val[k] = vals[p];
            k++;
        }
        rowptr[i + 1] = k;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* SELL-C-sigma of a CSR matrix.  Rows are stably sorted by descending length
 * inside consecutive windows of sigma rows; perm[new] = old.  Chunk c holds
 * sorted rows [cC, (c+1)C); its length is the longest row in it; storage is
 * column-major inside the chunk (entry j of local row r at ptr[c] + j C + r).
 * Padding: value +0.0, column = the row's own original index; slots of rows
 * past D hold column 0.                                                    */
int64_t orc_sell_size(int64_t D, const int64_t *rowptr, int C, int sigma,
                      int32_t *perm, int64_t *chunk_ptr, int32_t *chunk_len)
{
    if (C < 1 || sigma < 1) return -1;
    for (int64_t i = 0; i < D; i++) perm[i] = (int32_t)i;
    for (int64_t w = 0; w < D; w += sigma) {
        int64_t end = w + sigma < D ? w + sigma : D;
        /* stable insertion sort by descending length */
        for (int64_t p = w + 1; p < end; p++) {
            int32_t r = perm[p];
            int64_t len = rowptr[r + 1] - rowptr[r];
            int64_t q = p - 1;
            while (q >= w && (rowptr[perm[q] + 1] - rowptr[perm[q]]) < len) {
                perm[q + 1] = perm[q];
                q--;
            }
            perm[q + 1] = r;
        }
    }
    int64_t nchunks = (D + C - 1) / C;
    chunk_ptr[0] = 0;
    for (int64_t c = 0; c < nchunks; c++) {
        int64_t mx = 0;
        for (int r = 0; r < C; r++) {
            int64_t s = c * C + r;
            if (s < D) {
                int64_t len = rowptr[perm[s] + 1] - rowptr[perm[s]];
                if (len > mx) mx = len;
            }
        }
        chunk_len[c] = (int32_t)mx;
        chunk_ptr[c + 1] = chunk_ptr[c] + mx * C;
    }
    return chunk_ptr[nchunks];
}

void orc_sell_fill(int64_t D, const int64_t *rowptr, const uint32_t *col,
                   const double *val, int C, const int32_t *perm,
                   const int64_t *chunk_ptr, const int32_t *chunk_len,
                   uint32_t *scol, double *sval)
{
    int64_t nchunks = (D + C - 1) / C;
    for (int64_t c = 0; c < nchunks; c++) {
        for (int r = 0; r < C; r++) {
            int64_t s = c * C + r;
            for (int j = 0; j < chunk_len[c]; j++) {
                int64_t at = chunk_ptr[c] + (int64_t)j * C + r;
                if (s >= D) {
                    scol[at] = 0;
                    sval[at] = 0.0;
                    continue;
                }
                int64_t o = perm[s];
                int64_t len = rowptr[o + 1] - rowptr[o];
                if (j < len) {
                    scol[at] = col[rowptr[o] + j];
                    sval[at] = val[rowptr[o] + j];
                } else {
                    scol[at] = (uint32_t)o;
                    sval[at] = 0.0;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* STREAM triad c = a + s b (Sec. 3.2 measures b_m with STREAM).           */
void orc_triad(int64_t n, const double *a, const double *b, double *c, double s)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) c[i] = a[i] + s * b[i];
}

/* ------------------------------------------------------------------------ */
/* y = A x on row-major blocks: y[i*ldy + c] = sum_k val[k] x[col[k]*ldx + c]
 * (Eq. SpMVprocess applied to each of the nb vectors).                     */
void orc_spmmv(int64_t D, const int64_t *rowptr, const uint32_t *col,
               const double *val, int nb, const double *x, int64_t ldx,
               double *y, int64_t ldy)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; i++) {
        for (int c = 0; c < nb; c++) {
            double s = 0.0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++)
                s += val[k] * x[(int64_t)col[k] * ldx + c];
            y[i * ldy + c] = s;
        }
    }
}

/* Gershgorin discs: lo = min_i (a_ii - sum_{j!=i} |a_ij|), hi likewise.   */
void orc_gershgorin(int64_t D, const int64_t *rowptr, const uint32_t *col,
                    const double *val, double *lo, double *hi)
{
    double l = INFINITY, h = -INFINITY;
    for (int64_t i = 0; i < D; i++) {
        double d = 0.0, r = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) {
            if ((int64_t)col[k] == i) d += val[k];
            else r += fabs(val[k]);
        }
        if (d - r < l) l = d - r;
        if (d + r > h) h = d + r;
    }
    *lo = l;
    *hi = h;
}

/* ------------------------------------------------------------------------ */
/* Polynomial filter V <- sum_{k=0}^{n} mu_k T_k(B) V with B = alpha A + beta,
 * by the Chebyshev recurrence T_0 = I, T_1 = B, T_{k+1} = 2 B T_k - T_{k-1}.
 * Every step is a separate plain pass: SpMMV, then the vector updates.
 * T0, T1, T2 and AX are caller-provided D x nb scratch blocks (ld = nb).
 * Returns the number of SpMMVs performed (n).                              */
int orc_cheb_filter(int64_t D, const int64_t *rowptr, const uint32_t *col,
                    const double *val, int nb, double *V, int64_t ldv,
                    const double *mu, int n, double alpha, double beta,
                    double *T0, double *T1, double *T2, double *AX)
{
    int spmv = 0;
    if (n < 2) return -1;
    for (int64_t i = 0; i < D; i++)
        for (int c = 0; c < nb; c++) T0[i * nb + c] = V[i * ldv + c];
    /* T1 = alpha A T0 + beta T0 */
    orc_spmmv(D, rowptr, col, val, nb, T0, nb, AX, nb);
    spmv++;
    for (int64_t i = 0; i < D * nb; i++) T1[i] = alpha * AX[i] + beta * T0[i];
    /* V = mu_0 T0 + mu_1 T1 */
    for (int64_t i = 0; i < D; i++)
        for (int c = 0; c < nb; c++)
            V[i * ldv + c] = mu[0] * T0[i * nb + c] + mu[1] * T1[i * nb + c];
    for (int k = 2; k <= n; k++) {
        orc_spmmv(D, rowptr, col, val, nb, T1, nb, AX, nb);
        spmv++;
        for (int64_t i = 0; i < D * nb; i++)
            T2[i] = 2.0 * (alpha * AX[i] + beta * T1[i]) - T0[i];
        for (int64_t i = 0; i < D; i++)
            for (int c = 0; c < nb; c++) V[i * ldv + c] += mu[k] * T2[i * nb + c];
        double *tmp = T0;
        T0 = T1;
        T1 = T2;
        T2 = tmp;
    }
    return spmv;
}

/* ------------------------------------------------------------------------ */
/* Chebyshev coefficients of the indicator of [a, b] within [-1, 1]:
 *   c_0 = (acos a - acos b) / pi,
 *   c_k = 2 (sin(k acos a) - sin(k acos b)) / (k pi),
 * i.e. c_k = (2 - delta_k0)/pi * integral_{acos b}^{acos a} cos(k theta) dtheta.
 * Jackson damping for N = n + 1 moments (Weisse, Wellein, Alvermann,
 * Fehske, RMP 2006):
 *   g_k = [(N - k + 1) cos(pi k/(N+1)) + sin(pi k/(N+1)) cot(pi/(N+1))]/(N+1).
 * kind 0: window [a, b];  kind 1: Jackson-damped delta at a (b unused):
 *   mu_k = (2 - delta_k0) g_k T_k(a),  T_k(a) = cos(k acos a).              */
double orc_jackson(int n, int k)
{
    double N = (double)n + 1.0;
    double q = M_PI / (N + 1.0);
    return ((N - k + 1.0) * cos(q * k) + sin(q * k) * cos(q) / sin(q)) / (N + 1.0);
}

int orc_cheb_coeffs(int kind, double a, double b, int n, double *mu)
{
    if (n < 0 || a < -1.0 || a > 1.0) return 1;
    if (kind == 0) {
        if (b < a || b > 1.0) return 1;
        double ta = acos(a), tb = acos(b);
        for (int k = 0; k <= n; k++) {
            double c = (k == 0) ? (ta - tb) / M_PI
                                : 2.0 * (sin(k * ta) - sin(k * tb)) / (k * M_PI);
            mu[k] = orc_jackson(n, k) * c;
        }
        return 0;
    }
    if (kind == 1) {
        double ta = acos(a);
        for (int k = 0; k <= n; k++)
            mu[k] = (k == 0 ? 1.0 : 2.0) * orc_jackson(n, k) * cos(k * ta);
        return 0;
    }
    return 1;
}
