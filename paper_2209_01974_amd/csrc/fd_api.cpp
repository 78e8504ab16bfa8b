// libfd C ABI: handles, argument checks, the Chebyshev filter loop, the
// orthogonalization and Rayleigh-Ritz steps and the FD driver.
#include <atomic>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fd_internal.h"

namespace fd {

namespace {
thread_local std::string g_err;
}

fd_status fail(fd_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

fd_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? FD_ERR_OOM : FD_ERR_HIP;
}

namespace {

int vec_width(fd_dtype dt, int nb) {
    const int w = (dt == FD_F64) ? 2 : 4;
    return std::min(w, nb);
}

bool nb_ok(int nb) {
    return nb == 1 || nb == 2 || nb == 4 || nb == 8 || nb == 16 || nb == 32 || nb == 64;
}

size_t esize(fd_dtype dt) { return dt == FD_F64 ? 8 : 4; }

fd_status check_block(const void *p, int64_t ld, int64_t cols, fd_dtype dt, int nb, const char *name) {
    if (!p) return fail(FD_ERR_INVALID, std::string(name) + ": null pointer");
    if (ld < cols) return fail(FD_ERR_INVALID, std::string(name) + ": leading dimension smaller than width");
    const int vw = vec_width(dt, nb);
    if (ld % vw) return fail(FD_ERR_INVALID, std::string(name) + ": leading dimension not a multiple of the vector width");
    if (((uintptr_t)p) % (vw * esize(dt))) return fail(FD_ERR_INVALID, std::string(name) + ": misaligned");
    return FD_OK;
}

bool overlap(const void *a, int64_t la, const void *b, int64_t lb, int64_t D, size_t es) {
    const char *a0 = (const char *)a, *a1 = a0 + (size_t)D * la * es;
    const char *b0 = (const char *)b, *b1 = b0 + (size_t)D * lb * es;
    return a0 < b1 && b0 < a1;
}

// the same for blocks of wa and wb columns: the last row ends after its own
// columns, not after a full leading dimension
bool overlap_w(const void *a, int64_t la, int64_t wa, const void *b, int64_t lb, int64_t wb, int64_t D, size_t es) {
    if (D < 1) return false;
    const char *a0 = (const char *)a, *a1 = a0 + (size_t)((D - 1) * la + wa) * es;
    const char *b0 = (const char *)b, *b1 = b0 + (size_t)((D - 1) * lb + wb) * es;
    return a0 < b1 && b0 < a1;
}

template <typename T>
fd_status to_device(T **dst, const std::vector<T> &src) {
    FD_HIP(hipMalloc((void **)dst, std::max<size_t>(1, src.size()) * sizeof(T)));
    if (!src.empty()) FD_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return FD_OK;
}

// matrix-free Hubbard: the hop tables and spin masks, FP64 and FP32 elements
fd_status upload_tables(fd_matrix m) {
    DevMatrix &d = m->dev;
    const HubbardTables &T = m->hub;
    d.matfree = true;
    d.D = T.nu * T.nd;
    d.nu = T.nu;
    d.nd = T.nd;
    d.U = T.U;
    d.mf_maxu = d.mf_maxd = 0;
    for (size_t i = 0; i + 1 < T.off_u.size(); i++) d.mf_maxu = std::max(d.mf_maxu, T.off_u[i + 1] - T.off_u[i]);
    for (size_t i = 0; i + 1 < T.off_d.size(); i++) d.mf_maxd = std::max(d.mf_maxd, T.off_d[i + 1] - T.off_d[i]);
    std::vector<float> u32(T.val_u.begin(), T.val_u.end()), d32(T.val_d.begin(), T.val_d.end());
    FD_TRY(to_device(&d.mu, T.mu));
    FD_TRY(to_device(&d.md, T.md));
    FD_TRY(to_device(&d.off_u, T.off_u));
    FD_TRY(to_device(&d.off_d, T.off_d));
    FD_TRY(to_device(&d.idx_u, T.idx_u));
    FD_TRY(to_device(&d.idx_d, T.idx_d));
    FD_TRY(to_device(&d.val_u64, T.val_u));
    FD_TRY(to_device(&d.val_d64, T.val_d));
    FD_TRY(to_device(&d.val_u32, u32));
    FD_TRY(to_device(&d.val_d32, d32));
    // packed down hops for the LDS-staged pass: 15-bit targets and one
    // shared magnitude (the ring's hops are all +-t)
    bool pack = T.nd <= 32767 && !T.val_d.empty();
    const double tmag = pack ? std::fabs(T.val_d[0]) : 0.0;
    for (size_t i = 0; pack && i < T.val_d.size(); i++) pack = std::fabs(T.val_d[i]) == tmag && T.val_d[i] != 0.0;
    if (pack) {
        std::vector<uint16_t> h16(T.idx_d.size());
        for (size_t i = 0; i < h16.size(); i++)
            h16[i] = (uint16_t)(T.idx_d[i] | (T.val_d[i] > 0.0 ? 0x8000 : 0));
        FD_TRY(to_device(&d.hop16_d, h16));
        d.tmag_d = tmag;
    }
    FD_HIP(hipGetDevice(&m->device));
    return FD_OK;
}

fd_status upload(fd_matrix m) {
    if (m->fmt == FD_FMT_MATFREE) return upload_tables(m);
    DevMatrix &d = m->dev;
    const int64_t D = m->csr.D;
    d.D = D;
    std::vector<uint32_t> ptr;
    const std::vector<uint32_t> *col;
    const std::vector<double> *val;
    std::vector<int32_t> perm;
    if (m->fmt == FD_FMT_CSR) {
        if (m->csr.rowptr[D] >= (int64_t)UINT32_MAX) return fail(FD_ERR_UNSUPPORTED, "matrix: more than 2^32 entries");
        d.cshift = 0;
        d.nslots = D;
        d.stored = m->csr.rowptr[D];
        ptr.assign(m->csr.rowptr.begin(), m->csr.rowptr.end());
        col = &m->csr.col;
        val = &m->csr.val;
    } else {
        const HostSELL &S = m->sell;
        const int64_t nch = (int64_t)S.chunk_len.size();
        if (S.chunk_ptr[nch] >= (int64_t)UINT32_MAX) return fail(FD_ERR_UNSUPPORTED, "matrix: more than 2^32 slots");
        d.cshift = __builtin_ctz(S.C);
        d.nslots = nch * S.C;
        d.stored = S.chunk_ptr[nch];
        ptr.assign(S.chunk_ptr.begin(), S.chunk_ptr.end());
        col = &S.col;
        val = &S.val;
        perm.assign(d.nslots, -1);
        std::copy(S.perm.begin(), S.perm.end(), perm.begin());
    }
    d.maxlen = 0;
    d.minlen = INT32_MAX;
    for (size_t c = 0; c + 1 < ptr.size(); c++) {
        const int32_t len = (int32_t)((ptr[c + 1] - ptr[c]) >> d.cshift);
        d.maxlen = std::max<int32_t>(d.maxlen, len);
        d.minlen = std::min<int32_t>(d.minlen, len);
    }
    if (d.minlen > d.maxlen) d.minlen = d.maxlen;
    std::vector<float> v32(val->size());
    for (size_t i = 0; i < val->size(); i++) v32[i] = (float)(*val)[i];
    const size_t st = std::max<size_t>(1, (size_t)d.stored);
    FD_HIP(hipMalloc(&d.ptr, ptr.size() * sizeof(uint32_t)));
    FD_HIP(hipMalloc(&d.col, st * sizeof(uint32_t)));
    FD_HIP(hipMalloc(&d.val64, st * sizeof(double)));
    FD_HIP(hipMalloc(&d.val32, st * sizeof(float)));
    FD_HIP(hipMemcpy(d.ptr, ptr.data(), ptr.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    FD_HIP(hipMemcpy(d.col, col->data(), col->size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    FD_HIP(hipMemcpy(d.val64, val->data(), val->size() * sizeof(double), hipMemcpyHostToDevice));
    FD_HIP(hipMemcpy(d.val32, v32.data(), v32.size() * sizeof(float), hipMemcpyHostToDevice));
    if (!perm.empty()) {
        FD_HIP(hipMalloc(&d.perm, perm.size() * sizeof(int32_t)));
        FD_HIP(hipMemcpy(d.perm, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    FD_HIP(hipGetDevice(&m->device));
    return FD_OK;
}

void free_dev(DevMatrix &d) {
    if (d.ptr) (void)hipFree(d.ptr);
    if (d.col) (void)hipFree(d.col);
    if (d.val64) (void)hipFree(d.val64);
    if (d.val32) (void)hipFree(d.val32);
    if (d.perm) (void)hipFree(d.perm);
    void *tabs[] = {d.mu, d.md, d.off_u, d.off_d, d.idx_u, d.idx_d, d.val_u64, d.val_d64, d.val_u32, d.val_d32,
                    d.hop16_d};
    for (void *p : tabs)
        if (p) (void)hipFree(p);
    d = DevMatrix();
}

fd_status need_device(fd_matrix m) {
    if (!m) return fail(FD_ERR_INVALID, "null matrix handle");
    if (m->device < 0) return fail(FD_ERR_INVALID, "matrix was built host-only");
    return FD_OK;
}

// The filter on one group of bundles (all at once, or one at a time).
fd_status filter_run(const DevMatrix &M, fd_dtype dt, int nb, int nbund, char *V, int64_t ldv,
                     const double *mu, int degree, double alpha, double beta, char *W1, char *W2,
                     int64_t ldw, int64_t bw, hipStream_t s) {
    const size_t es = esize(dt);
    (void)es;
    SpmmvCall c;
    c.nb = nb;
    c.nbundles = nbund;
    // step 1: W2 = T_1 V = alpha A V + beta V
    c.mode = 1;
    c.x = V; c.ldx = ldv; c.bx = nb;
    c.y = W2; c.ldy = ldw; c.by = bw;
    c.a = alpha; c.b = beta;
    FD_TRY(launch_spmmv(M, dt, c, s));
    // step 2: W1 = T_2 V = 2 B W2 - V;  V = mu0 V + mu1 W2 + mu2 W1
    c.mode = 2;
    c.x = W2; c.ldx = ldw; c.bx = bw;
    c.y = W1; c.ldy = ldw; c.by = bw;
    c.v = V; c.ldv = ldv; c.bv = nb;
    c.a = 2.0 * alpha; c.b = 2.0 * beta;
    c.cv = mu[0]; c.cx = mu[1]; c.ct = mu[2];
    FD_TRY(launch_spmmv(M, dt, c, s));
    // steps k >= 3: prev = 2 B cur - prev (in place).  V is updated every
    // other step with two terms, V += mu_{k-1} cur + mu_k prev at even k
    // (cur's own row is read by the step anyway), which saves one read and
    // one write of V per pair of steps; an odd last step adds mu_n alone.
    char *cur = W1, *prev = W2;
    for (int k = 3; k <= degree; k++) {
        c.x = cur; c.ldx = ldw; c.bx = bw;
        c.z = prev; c.ldz = ldw; c.bz = bw;
        c.y = prev; c.ldy = ldw; c.by = bw;
        if (k % 2 == 0) {
            c.mode = 5;
            c.cx = mu[k - 1];
            c.ct = mu[k];
        } else if (k == degree) {
            c.mode = 3;
            c.ct = mu[k];
        } else {
            c.mode = 4;
        }
        FD_TRY(launch_spmmv(M, dt, c, s));
        std::swap(cur, prev);
    }
    return FD_OK;
}

fd_status cheb_filter_impl(fd_matrix m, fd_dtype dt, int nb, int nbund, void *V, int64_t ldv,
                           const double *mu, int degree, double alpha, double beta, void *W1, void *W2,
                           int64_t ldw, hipStream_t s) {
    const DevMatrix &M = m->dev;
    const size_t es = esize(dt);
    if (ldw >= (int64_t)nb * nbund) {
        return filter_run(M, dt, nb, nbund, (char *)V, ldv, mu, degree, alpha, beta, (char *)W1, (char *)W2,
                          ldw, nb, s);
    }
    // One bundle after another.  When V is wider than a bundle, each bundle
    // is staged in a contiguous D x nb slab (a gather and a scatter per
    // filter application) so that the degree steps stream V contiguously.
    char *stage = nullptr;
    if (ldv != nb && degree >= 8) stage = (char *)workspace((size_t)M.D * nb * es, 7);
    for (int b = 0; b < nbund; b++) {
        char *Vb = (char *)V + (size_t)b * nb * es;
        if (stage) {
            FD_TRY(copy_rows(M.D, (int64_t)nb * es, Vb, ldv * (int64_t)es, stage, (int64_t)nb * es, s));
            FD_TRY(filter_run(M, dt, nb, 1, stage, nb, mu, degree, alpha, beta, (char *)W1, (char *)W2, ldw, 0, s));
            FD_TRY(copy_rows(M.D, (int64_t)nb * es, stage, (int64_t)nb * es, Vb, ldv * (int64_t)es, s));
        } else {
            FD_TRY(filter_run(M, dt, nb, 1, Vb, ldv, mu, degree, alpha, beta, (char *)W1, (char *)W2, ldw, 0, s));
        }
    }
    return FD_OK;
}

// ---------------------------------------------------------- small buffers --
struct Small {
    double *G, *Q, *work, *theta, *rho, *E;
    int *keep, *ints;
};

fd_status small_buffers(int n, Small &b) {
    const size_t nn = (size_t)n * n;
    const size_t bytes = (4 * nn + (2 * n + nn) + 2 * n) * sizeof(double) + (n + 8) * sizeof(int);
    char *p = (char *)workspace(bytes, 3);
    if (!p) return fail(FD_ERR_OOM, "small workspace");
    b.G = (double *)p;
    b.Q = b.G + nn;
    b.work = b.Q + nn;
    b.theta = b.work + 2 * n + nn;
    b.rho = b.theta + n;
    b.E = b.rho + n;  // two n x n matrices
    b.keep = (int *)(b.E + 2 * nn);
    b.ints = b.keep + n;
    return FD_OK;
}

fd_status orthog_impl(int64_t D, int ns, double *V, int64_t ldv, int method, uint64_t seed, int *rank_out,
                      hipStream_t s) {
    Small b;
    FD_TRY(small_buffers(ns, b));
    if (method == FD_ORTHO_CHOLQR2) {
        bool ok = true;
        for (int pass = 0; pass < 2 && ok; pass++) {
            FD_TRY(gram(D, ns, ns, V, ldv, V, ldv, b.G, ns, true, s));
            FD_TRY(cholqr_transform(ns, b.G, b.Q, b.ints, pass == 1, s));
            int okh = 0;
            FD_HIP(hipMemcpyAsync(&okh, b.ints, sizeof(int), hipMemcpyDeviceToHost, s));
            FD_HIP(hipStreamSynchronize(s));
            ok = okh != 0;
            if (ok) FD_TRY(rotate(D, ns, ns, V, ldv, b.Q, ns, s));
        }
        if (ok) {
            if (rank_out) *rank_out = ns;
            return FD_OK;
        }
        // fall through to SVQB2 on the partly orthogonalized block
    }
    int rank = ns;
    FD_TRY(gram(D, ns, ns, V, ldv, V, ldv, b.G, ns, true, s));
    FD_TRY(svqb_transform(ns, b.G, b.Q, b.work, b.keep, b.ints, s));
    FD_TRY(rotate(D, ns, ns, V, ldv, b.Q, ns, s));
    FD_HIP(hipMemcpyAsync(&rank, b.ints, sizeof(int), hipMemcpyDeviceToHost, s));
    FD_HIP(hipStreamSynchronize(s));
    if (rank < 0) return fail(FD_ERR_BREAKDOWN, "orthogonalization: non-finite Gram matrix");
    if (rank < ns) {
        // replace the directions that were clipped by fresh random vectors
        FD_TRY(refill_random(D, ns, V, ldv, b.keep, seed, s));
        FD_TRY(gram(D, ns, ns, V, ldv, V, ldv, b.G, ns, true, s));
        FD_TRY(svqb_transform(ns, b.G, b.Q, b.work, b.keep, b.ints + 1, s));
        FD_TRY(rotate(D, ns, ns, V, ldv, b.Q, ns, s));
    }
    // Second pass.  One pass leaves V^t V = I + E with |E| about kappa eps;
    // when n max|E_ij| <= 1e-5 the pass takes Q = (I + E)^-1/2 from its
    // series (the orthonormal basis nearest V: the span, all the next
    // Rayleigh-Ritz step or filter depends on, is SVQB's), else SVQB again.
    FD_TRY(gram(D, ns, ns, V, ldv, V, ldv, b.G, ns, true, s));
    FD_TRY(lowdin_transform(ns, b.G, b.E, b.E + (size_t)ns * ns, b.Q, b.ints + 3, s));
    int okl = 0;
    FD_HIP(hipMemcpyAsync(&okl, b.ints + 3, sizeof(int), hipMemcpyDeviceToHost, s));
    FD_HIP(hipStreamSynchronize(s));
    if (!okl) FD_TRY(svqb_transform(ns, b.G, b.Q, b.work, b.keep, b.ints + 2, s));
    FD_TRY(rotate(D, ns, ns, V, ldv, b.Q, ns, s));
    if (rank_out) *rank_out = rank;
    return FD_OK;
}

// Rayleigh-Ritz once W = A V is in place: H = V^t W, H = Y Theta Y^t,
// V <- V Y, W <- W Y, rho_j = ||W_j - theta_j V_j||; theta and rho to the host.
fd_status rr_dense(int64_t D, int ns, double *V, double *W, int64_t ld, double *theta_host, double *resid_host,
                   hipStream_t s) {
    Small b;
    FD_TRY(small_buffers(ns, b));
    FD_TRY(gram(D, ns, ns, V, ld, W, ld, b.G, ns, false, s));
    FD_TRY(symmetrize(ns, b.G, s));
    FD_TRY(syev(ns, b.G, ns, b.theta, b.Q, ns, s));
    FD_TRY(rotate(D, ns, ns, V, ld, b.Q, ns, s));
    FD_TRY(rotate(D, ns, ns, W, ld, b.Q, ns, s));
    FD_TRY(col_resid(D, ns, V, W, ld, b.theta, b.rho, s));
    FD_HIP(hipMemcpyAsync(theta_host, b.theta, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    FD_HIP(hipMemcpyAsync(resid_host, b.rho, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    FD_HIP(hipStreamSynchronize(s));
    return FD_OK;
}

// Lehmann's method (Lehmann 1963; the paper takes its target and search
// intervals from Lehmann intervals, Sec. 2): the eigenvalues mu of the
// pencil S x = mu B x with S = V^t (A - rho) V and
// B = ((A - rho) V)^t ((A - rho) V), W = A V given.  B = R^t R (Cholesky),
// then mu = eig(R^-t S R^-1), ascending, to the host.
fd_status lehmann_impl(int64_t D, int n, const double *V, const double *W, int64_t ld, double rho,
                       double *mu_host, hipStream_t s) {
    const size_t nn = (size_t)n * n;
    char *ws = (char *)workspace((7 * nn + n) * sizeof(double) + 64, 8);
    if (!ws) return fail(FD_ERR_OOM, "Lehmann: workspace");
    double *G2 = (double *)ws, *G1 = G2 + nn, *G0 = G1 + nn, *B = G0 + nn, *S = B + nn, *Q = S + nn, *C = Q + nn;
    double *mu = C + nn;
    int *ok = (int *)(mu + n);
    FD_TRY(gram(D, n, n, W, ld, W, ld, G2, n, true, s));
    FD_TRY(gram(D, n, n, V, ld, W, ld, G1, n, false, s));
    FD_TRY(gram(D, n, n, V, ld, V, ld, G0, n, true, s));
    FD_TRY(lehmann_pencil(n, G2, G1, G0, rho, B, S, s));
    FD_TRY(cholqr_transform(n, B, Q, ok, false, s));
    int okh = 0;
    FD_HIP(hipMemcpyAsync(&okh, ok, sizeof(int), hipMemcpyDeviceToHost, s));
    FD_HIP(hipStreamSynchronize(s));
    if (!okh)
        return fail(FD_ERR_BREAKDOWN, "Lehmann: (A - rho) V is rank deficient (rho an eigenvalue with its vector in V?)");
    FD_TRY(rotate(n, n, n, S, n, Q, n, s));                 // S <- S R^-1
    FD_TRY(gram(n, n, n, Q, n, S, n, C, n, false, s));      // C = R^-t S R^-1
    FD_TRY(symmetrize(n, C, s));
    FD_TRY(syev(n, C, n, mu, G2, n, s));
    FD_HIP(hipMemcpyAsync(mu_host, mu, n * sizeof(double), hipMemcpyDeviceToHost, s));
    FD_HIP(hipStreamSynchronize(s));
    return FD_OK;
}

// Lehmann radius: the smallest r such that [rho - r, rho + r] provably
// holds at least k eigenvalues (interval counts of both sides add up, since
// [rho + 1/mu_i, rho) and (rho, rho + 1/mu_j] are disjoint).  INFINITY if
// the subspace certifies fewer than k.
double lehmann_radius(const std::vector<double> &mu, int k) {
    std::vector<double> d;
    for (double x : mu)
        if (x != 0.0) d.push_back(std::fabs(1.0 / x));
    std::sort(d.begin(), d.end());
    return (int)d.size() >= k ? d[k - 1] : INFINITY;
}

fd_status rr_impl(fd_matrix m, int ns, int nb, double *V, double *W, int64_t ld, double *theta_host,
                  double *resid_host, hipStream_t s) {
    SpmmvCall c;
    c.mode = 0;
    c.nb = nb;
    c.nbundles = ns / nb;
    c.x = V; c.ldx = ld; c.bx = nb;
    c.y = W; c.ldy = ld; c.by = nb;
    FD_TRY(launch_spmmv(m->dev, FD_F64, c, s));
    return rr_dense(m->dev.D, ns, V, W, ld, theta_host, resid_host, s);
}

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// FD_TRACE=1: the solvers write one JSON line per outer iteration to
// stderr; FD_TRACE_FILE: the same lines appended to that file (flushed line
// by line)
bool trace_on() {
    const char *tr = std::getenv("FD_TRACE");
    const char *trf = std::getenv("FD_TRACE_FILE");
    return (tr && tr[0] == '1') || (trf && trf[0]);
}

void trace_line(const char *line) {
    const char *tr = std::getenv("FD_TRACE");
    const char *trf = std::getenv("FD_TRACE_FILE");
    if (tr && tr[0] == '1') {
        std::fputs(line, stderr);
        std::fflush(stderr);
    }
    if (trf && trf[0]) {
        if (FILE *f = std::fopen(trf, "a")) {
            std::fputs(line, f);
            std::fclose(f);
        }
    }
}

// Ritz values in the window nearest tau (ties: lower value first).
std::vector<int> select_targets(const std::vector<double> &th, double lo, double hi, int nt) {
    const double tau = 0.5 * (lo + hi);
    std::vector<int> idx;
    for (int j = 0; j < (int)th.size(); j++)
        if (hi <= lo || (th[j] >= lo && th[j] <= hi)) idx.push_back(j);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        const double da = std::fabs(th[a] - tau), db = std::fabs(th[b] - tau);
        if (da != db) return da < db;
        return th[a] < th[b];
    });
    if ((int)idx.size() > nt) idx.resize(nt);
    return idx;
}

// KPM counting function: estimated number of eigenvalues in tau +- r
double kpm_count(const std::vector<double> &mu, int64_t D, double alpha, double beta, double lo, double hi) {
    const int M = (int)mu.size();
    std::vector<double> c(M);
    const double a = std::max(-1.0, std::min(1.0, alpha * lo + beta));
    const double b = std::max(a, std::min(1.0, alpha * hi + beta));
    if (cheb_coeffs(0, a, b, M - 1, c.data()) != FD_OK) return 0.0;
    double n = 0.0;
    for (int k = 0; k < M; k++) n += c[k] * mu[k];
    return n * (double)D;
}

// smallest radius r (bisection) with count(tau +- r, clipped to [lo, hi]) >= want
double kpm_radius(const std::vector<double> &mu, int64_t D, double alpha, double beta, double tau, double lo,
                  double hi, double want) {
    double r0 = 0.0, r1 = std::max(tau - lo, hi - tau);
    if (kpm_count(mu, D, alpha, beta, lo, hi) < want) return r1;
    for (int it = 0; it < 60; it++) {
        const double r = 0.5 * (r0 + r1);
        if (kpm_count(mu, D, alpha, beta, std::max(lo, tau - r), std::min(hi, tau + r)) >= want) r1 = r;
        else r0 = r;
    }
    return r1;
}

// Test hook: device buffers of the solvers larger than this many bytes fail
// as if the device were out of memory (0: no limit).
std::atomic<int64_t> g_alloc_limit{0};

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    fd_status alloc(size_t bytes, const char *what) {
        const int64_t lim = g_alloc_limit.load();
        if (lim > 0 && (int64_t)bytes > lim)
            return fail(FD_ERR_OOM, std::string("cannot allocate ") + what + " (allocation limit set)");
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(FD_ERR_OOM, std::string("cannot allocate ") + what);
        }
        return FD_OK;
    }
};

// k steps of Lanczos with full reorthogonalization (classical Gram-Schmidt
// against every earlier basis vector, twice) from the seeded start vector
// (Sec. 2: the spectral bounds come from a few Lanczos steps).  Stops early
// when the new vector's norm drops to 1e-12 of the largest |alpha|
// (invariant subspace).  theta: Ritz values of the tridiagonal, ascending;
// resid: their residual bounds beta_k |s_kj|.  Synchronizes.
// M's rows gather x at the row indices M.col, shifted by -xoff (a slice of a
// block-diagonal stack whose columns carry the slice's first row).
fd_status lanczos_impl(const DevMatrix &M, int64_t xoff, int k, uint64_t seed, std::vector<double> &theta,
                       std::vector<double> &resid, hipStream_t s) {
    const int64_t D = M.D;
    if (k < 1 || k > 512) return fail(FD_ERR_INVALID, "Lanczos: need 1 <= k <= 512");
    k = (int)std::min<int64_t>(k, D);
    const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (D + 8191) / 8192));
    DevBuf Q;
    FD_TRY(Q.alloc((size_t)(k + 1) * D * 8, "the Lanczos basis"));
    double *Qd = (double *)Q.p;
    // small device buffers: c (k, first Gram-Schmidt pass), c2 (k, second
    // pass), c3 (1, squared norm) in a row, partial sums (nblk k), T (k k),
    // U (k k), w (k)
    const size_t nsmall = 2 * (size_t)k + 1 + (size_t)nblk * k + 2 * (size_t)k * k + k;
    double *c = (double *)workspace(nsmall * sizeof(double), 9);
    if (!c) return fail(FD_ERR_OOM, "Lanczos: workspace");
    double *c2 = c + k, *c3 = c2 + k;
    double *P = c3 + 1, *T = P + (size_t)nblk * k, *U = T + (size_t)k * k, *w = U + (size_t)k * k;
    std::vector<double> hb(2 * (size_t)k + 1);
    auto norm_of = [&](const double *v, double &out) -> fd_status {
        FD_TRY(lz_dots(D, 1, v, v, c, P, nblk, s));
        double h = 0.0;
        FD_HIP(hipMemcpyAsync(&h, c, sizeof(double), hipMemcpyDeviceToHost, s));
        FD_HIP(hipStreamSynchronize(s));
        out = std::sqrt(h);
        return FD_OK;
    };
    FD_TRY(lz_start(D, Qd, seed, s));
    double b0 = 0.0;
    FD_TRY(norm_of(Qd, b0));
    if (!(b0 > 0.0)) return fail(FD_ERR_BREAKDOWN, "Lanczos: zero start vector");
    FD_TRY(lz_scale(D, Qd, 1.0 / b0, s));
    std::vector<double> alpha(k, 0.0), beta(k, 0.0);
    int steps = k;
    for (int j = 0; j < k; j++) {
        double *qj = Qd + (int64_t)j * D, *wv = Qd + (int64_t)(j + 1) * D;
        SpmmvCall call;
        call.mode = 0;
        call.nb = 1;
        call.x = qj - xoff;
        call.ldx = 1;
        call.y = wv;
        call.ldy = 1;
        FD_TRY(launch_spmmv(M, FD_F64, call, s));
        // two Gram-Schmidt passes (coefficients in c, then c2) and the norm
        // (c3); one read-back per step: c[j], c2[j] and c3 lie in one range
        FD_TRY(lz_dots(D, j + 1, Qd, wv, c, P, nblk, s));
        FD_TRY(lz_sub(D, j + 1, Qd, c, wv, s));
        FD_TRY(lz_dots(D, j + 1, Qd, wv, c2, P, nblk, s));
        FD_TRY(lz_sub(D, j + 1, Qd, c2, wv, s));
        FD_TRY(lz_dots(D, 1, wv, wv, c3, P, nblk, s));
        const size_t nrd = 2 * (size_t)k + 1 - (size_t)j;
        FD_HIP(hipMemcpyAsync(hb.data() + j, c + j, nrd * sizeof(double), hipMemcpyDeviceToHost, s));
        FD_HIP(hipStreamSynchronize(s));
        alpha[j] += hb[j];
        alpha[j] += hb[k + j];
        beta[j] = std::sqrt(hb[2 * (size_t)k]);
        double amax = 0.0;
        for (int i = 0; i <= j; i++) amax = std::max(amax, std::fabs(alpha[i]));
        if (!std::isfinite(beta[j]) || !std::isfinite(alpha[j]))
            return fail(FD_ERR_BREAKDOWN, "Lanczos: non-finite recurrence");
        if (beta[j] <= 1e-12 * amax) {
            steps = j + 1;
            break;
        }
        FD_TRY(lz_scale(D, wv, 1.0 / beta[j], s));
    }
    std::vector<double> Th((size_t)steps * steps, 0.0);
    for (int i = 0; i < steps; i++) {
        Th[(size_t)i * steps + i] = alpha[i];
        if (i + 1 < steps) Th[(size_t)i * steps + i + 1] = Th[(size_t)(i + 1) * steps + i] = beta[i];
    }
    FD_HIP(hipMemcpyAsync(T, Th.data(), Th.size() * sizeof(double), hipMemcpyHostToDevice, s));
    FD_TRY(syev(steps, T, steps, w, U, steps, s));
    theta.assign(steps, 0.0);
    std::vector<double> Uh((size_t)steps * steps);
    FD_HIP(hipMemcpyAsync(theta.data(), w, steps * sizeof(double), hipMemcpyDeviceToHost, s));
    FD_HIP(hipMemcpyAsync(Uh.data(), U, Uh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    FD_HIP(hipStreamSynchronize(s));
    resid.assign(steps, 0.0);
    for (int j = 0; j < steps; j++) resid[j] = beta[steps - 1] * std::fabs(Uh[(size_t)(steps - 1) * steps + j]);
    return FD_OK;
}

// ||H|| of the convergence test: the largest |Ritz value| of 40 Lanczos
// steps from SplitMix64 seed 1, a lower bound of ||H||_2, so that
// rho <= tol ||H|| is never looser than the target.  Cached in the handle.
constexpr int kNormSteps = 40;
constexpr uint64_t kNormSeed = 1;
fd_status lanczos_norm(fd_matrix m, double &out, hipStream_t s) {
    if (!(m->lz_norm >= 0.0)) {
        std::vector<double> th, rs;
        FD_TRY(lanczos_impl(m->dev, 0, kNormSteps, kNormSeed, th, rs, s));
        m->lz_norm = std::max(std::fabs(th.front()), std::fabs(th.back()));
    }
    out = m->lz_norm;
    return FD_OK;
}

}  // namespace
}  // namespace fd

// Batched problems: a block-diagonal stack of instance matrices on one device.
struct fd_batch_s {
    int device = -1;
    std::vector<int64_t> off;  // n_inst + 1 row offsets
    std::vector<double> lam_lo, lam_hi;
    std::vector<double> lz_norm;  // per instance ||H|| estimate (Lanczos), filled on first use
    fd::BatchDev dev;
    int32_t mu_cap = 0;  // entries allocated in dev.mu
    hipStream_t cap = nullptr;  // capture-only stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct Key {
        int dt = -1, nb = 0, nbund = 0, max_degree = 0, mstride = 0;
        const void *V = nullptr, *W1 = nullptr, *W2 = nullptr, *mu = nullptr;
        int64_t ldv = 0, ldw = 0;
        bool operator==(const Key &o) const {
            return dt == o.dt && nb == o.nb && nbund == o.nbund && max_degree == o.max_degree &&
                   mstride == o.mstride && V == o.V && W1 == o.W1 && W2 == o.W2 && mu == o.mu && ldv == o.ldv &&
                   ldw == o.ldw;
        }
    } key;
    int64_t graph_launches = 0, graph_captures = 0;
};

namespace fd {
namespace {

void batch_release(fd_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    BatchDev &d = b->dev;
    void *bufs[] = {d.ptr,   d.col,      d.val64,   d.val32,   d.inst,    d.alpha,   d.beta, d.deg,
                    d.act,   d.mu,       d.off,     d.seg_inst, d.inst_s0, d.rc_inst, d.seg_r0, d.seg_r1,
                    d.rc_r0};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    d = BatchDev();
    b->exec = nullptr;
    b->graph = nullptr;
    b->cap = nullptr;
}

// Per-instance filter parameters to the device (ordered on stream s).
fd_status batch_params(fd_batch b, const double *alpha, const double *beta, const int32_t *deg,
                       const int32_t *act, const double *mu, int32_t mstride, hipStream_t s) {
    BatchDev &d = b->dev;
    const int n = d.n_inst;
    if (mu && (int64_t)n * mstride > b->mu_cap) {
        FD_HIP(hipStreamSynchronize(s));
        if (d.mu) (void)hipFree(d.mu);
        d.mu = nullptr;
        b->mu_cap = 0;
        FD_HIP(hipMalloc(&d.mu, (size_t)n * mstride * sizeof(double)));
        b->mu_cap = n * mstride;
    }
    if (alpha) FD_HIP(hipMemcpyAsync(d.alpha, alpha, n * sizeof(double), hipMemcpyHostToDevice, s));
    if (beta) FD_HIP(hipMemcpyAsync(d.beta, beta, n * sizeof(double), hipMemcpyHostToDevice, s));
    if (deg) FD_HIP(hipMemcpyAsync(d.deg, deg, n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (act) FD_HIP(hipMemcpyAsync(d.act, act, n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (mu) {
        FD_HIP(hipMemcpyAsync(d.mu, mu, (size_t)n * mstride * sizeof(double), hipMemcpyHostToDevice, s));
        d.mstride = mstride;
    }
    // the host arrays may be temporaries of the caller
    FD_HIP(hipStreamSynchronize(s));
    return FD_OK;
}

// The degree steps of the filter on every instance (Alg. 2 caption): step 1
// W2 = T_1 V, step 2 W1 = T_2 V and V = mu_0 V + mu_1 W2 + mu_2 W1, steps
// k >= 3 prev = 2 B cur - prev in place and V += mu_k prev.  Each instance
// stops after its own degree.  All bundles in one launch per step.
fd_status batch_filter_steps(const BatchDev &B, fd_dtype dt, int nb, int nbund, char *V, int64_t ldv,
                             int max_degree, char *W1, char *W2, int64_t ldw, hipStream_t s) {
    BatchCall c;
    c.nb = nb;
    c.nbundles = nbund;
    c.mode = 1;
    c.k = 1;
    c.x = V; c.ldx = ldv; c.bx = nb;
    c.y = W2; c.ldy = ldw; c.by = nb;
    FD_TRY(launch_batch(B, dt, c, s));
    c.mode = 2;
    c.k = 2;
    c.x = W2; c.ldx = ldw; c.bx = nb;
    c.y = W1; c.ldy = ldw; c.by = nb;
    c.v = V; c.ldv = ldv; c.bv = nb;
    FD_TRY(launch_batch(B, dt, c, s));
    char *cur = W1, *prev = W2;
    for (int k = 3; k <= max_degree; k++) {
        c.mode = 5;  // V every other step, two terms (per-instance last step)
        c.k = k;
        c.x = cur; c.ldx = ldw; c.bx = nb;
        c.z = prev; c.ldz = ldw; c.bz = nb;
        c.y = prev; c.ldy = ldw; c.by = nb;
        FD_TRY(launch_batch(B, dt, c, s));
        std::swap(cur, prev);
    }
    return FD_OK;
}

// Run the steps eagerly, or as one replay of a HIP graph captured on the
// handle's private stream (re-captured when buffers, shape or degree change).
fd_status batch_filter_run(fd_batch b, fd_dtype dt, int nb, int nbund, char *V, int64_t ldv, int max_degree,
                           char *W1, char *W2, int64_t ldw, bool use_graph, hipStream_t s) {
    if (!use_graph) return batch_filter_steps(b->dev, dt, nb, nbund, V, ldv, max_degree, W1, W2, ldw, s);
    fd_batch_s::Key k;
    k.dt = (int)dt;
    k.nb = nb;
    k.nbund = nbund;
    k.max_degree = max_degree;
    k.V = V;
    k.W1 = W1;
    k.W2 = W2;
    k.ldv = ldv;
    k.ldw = ldw;
    k.mu = b->dev.mu;  // the kernels take these by value
    k.mstride = b->dev.mstride;
    if (!b->exec || !(k == b->key)) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        if (!b->cap) FD_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        FD_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        fd_status st = batch_filter_steps(b->dev, dt, nb, nbund, V, ldv, max_degree, W1, W2, ldw, b->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &g);
        if (st != FD_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "batched filter: graph capture");
        b->graph = g;
        FD_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->key = k;
        b->graph_captures++;
    }
    FD_HIP(hipGraphLaunch(b->exec, s));
    b->graph_launches++;
    return FD_OK;
}

}  // namespace
}  // namespace fd

using namespace fd;

extern "C" {

const char *fd_last_error(void) { return g_err.c_str(); }

fd_status fd_build_matrix(const fd_model_params *p, fd_format fmt, int32_t C, int32_t sigma, int32_t flags,
                          fd_matrix *out) {
    if (!p || !out) return fail(FD_ERR_INVALID, "fd_build_matrix: null argument");
    if (fmt != FD_FMT_CSR && fmt != FD_FMT_SELL && fmt != FD_FMT_MATFREE && fmt != FD_FMT_PENCIL)
        return fail(FD_ERR_INVALID, "fd_build_matrix: bad format");
    if (fmt == FD_FMT_PENCIL && p->model != FD_ANDERSON_3D)
        return fail(FD_ERR_INVALID, "fd_build_matrix: the pencil order is for the 3D Anderson lattice only");
    if (fmt == FD_FMT_MATFREE && p->model != FD_HUBBARD_RING)
        return fail(FD_ERR_INVALID, "fd_build_matrix: the matrix-free format is for the Hubbard ring only");
    if (fmt == FD_FMT_MATFREE && (C < 0 || C > (1 << 20)))
        return fail(FD_ERR_INVALID, "fd_build_matrix: matrix-free tile C must be in [0, 2^20]");
    fd_matrix m = new (std::nothrow) fd_matrix_s;
    if (!m) return fail(FD_ERR_OOM, "fd_build_matrix: host allocation");
    fd_status st;
    if (fmt == FD_FMT_MATFREE) {
        st = hubbard_tables(p->L, p->n_up, p->n_dn, p->periodic != 0, p->t, p->U, p->config_order, m->hub);
        m->fmt = fmt;
        if (st == FD_OK) {
            m->D = m->hub.nu * m->hub.nd;
            m->nnz = hubbard_tables_nnz(m->hub);
            m->stored = (int64_t)(m->hub.idx_u.size() + m->hub.idx_d.size());
            hubbard_tables_gershgorin(m->hub, m->lam_lo, m->lam_hi);
            m->dev.mf_tile = C > 0 ? C : 16;
        }
        if (st == FD_OK && !(flags & FD_BUILD_HOST_ONLY)) {
            st = upload(m);
            if (st != FD_OK) free_dev(m->dev);
        }
        if (st != FD_OK) {
            delete m;
            return st;
        }
        *out = m;
        return FD_OK;
    }
    switch (p->model) {
        case FD_HUBBARD_RING:
            st = build_hubbard(p->L, p->n_up, p->n_dn, p->periodic != 0, p->t, p->U, p->config_order, m->csr,
                               m->cfg_up, m->cfg_dn);
            break;
        case FD_ANDERSON_3D:
            if (p->tile_x < 0 || p->tile_y < 0 || (p->tile_x == 0) != (p->tile_y == 0))
                st = fail(FD_ERR_INVALID, "Anderson: tile_x and tile_y both 0 (natural numbering) or both >= 1");
            else if (p->tile_x > 0 && fmt == FD_FMT_PENCIL)
                st = fail(FD_ERR_INVALID, "Anderson: the pencil walk needs the natural site numbering");
            else
                st = build_anderson(p->L, p->t, p->W, p->seed, p->skip, m->csr);
            if (st == FD_OK && p->tile_x > 0) st = relabel_tiles(p->L, p->tile_x, p->tile_y, m->csr);
            break;
        case FD_DIAGONAL: st = build_diagonal(p->n, p->diag, m->csr); break;
        case FD_USER_CSR: st = build_user(p->D, p->rowptr, p->col, p->val, m->csr); break;
        default: st = fail(FD_ERR_INVALID, "fd_build_matrix: unknown model");
    }
    if (st == FD_OK && fmt == FD_FMT_SELL) st = build_sell(m->csr, C, sigma, m->sell);
    if (st == FD_OK && fmt == FD_FMT_PENCIL)
        st = build_pencil(m->csr, p->L, C > 0 ? C : 16, sigma > 0 ? sigma : 16, m->sell);
    m->fmt = fmt;
    if (st == FD_OK) {
        gershgorin(m->csr, m->lam_lo, m->lam_hi);
        m->D = m->csr.D;
        m->nnz = m->csr.rowptr[m->csr.D];
        m->stored = (fmt == FD_FMT_SELL || fmt == FD_FMT_PENCIL) ? m->sell.chunk_ptr.back() : m->nnz;
    }
    if (st == FD_OK && !(flags & FD_BUILD_HOST_ONLY)) {
        st = upload(m);
        if (st != FD_OK) free_dev(m->dev);
    }
    if (st != FD_OK) {
        delete m;
        return st;
    }
    *out = m;
    return FD_OK;
}

fd_status fd_matrix_info(fd_matrix m, int64_t *D, int64_t *nnz, int64_t *stored, double *lo, double *hi) {
    if (!m) return fail(FD_ERR_INVALID, "fd_matrix_info: null handle");
    if (D) *D = m->D;
    if (nnz) *nnz = m->nnz;
    if (stored) *stored = m->stored;
    if (lo) *lo = m->lam_lo;
    if (hi) *hi = m->lam_hi;
    return FD_OK;
}

fd_status fd_matrix_export_csr(fd_matrix m, int64_t *rowptr, uint32_t *col, double *val) {
    if (!m || !rowptr || !col || !val) return fail(FD_ERR_INVALID, "fd_matrix_export_csr: null argument");
    if (m->fmt == FD_FMT_MATFREE) return fail(FD_ERR_INVALID, "fd_matrix_export_csr: matrix-free matrix stores no CSR");
    std::memcpy(rowptr, m->csr.rowptr.data(), m->csr.rowptr.size() * sizeof(int64_t));
    std::memcpy(col, m->csr.col.data(), m->csr.col.size() * sizeof(uint32_t));
    std::memcpy(val, m->csr.val.data(), m->csr.val.size() * sizeof(double));
    return FD_OK;
}

fd_status fd_matrix_export_sell(fd_matrix m, int32_t *perm, int64_t *cptr, int32_t *clen, uint32_t *col,
                                double *val) {
    if (!m || !perm || !cptr || !clen || !col || !val)
        return fail(FD_ERR_INVALID, "fd_matrix_export_sell: null argument");
    if (m->fmt != FD_FMT_SELL && m->fmt != FD_FMT_PENCIL)
        return fail(FD_ERR_INVALID, "fd_matrix_export_sell: matrix is not SELL or pencil-ordered");
    const HostSELL &S = m->sell;
    std::memcpy(perm, S.perm.data(), S.perm.size() * sizeof(int32_t));
    std::memcpy(cptr, S.chunk_ptr.data(), S.chunk_ptr.size() * sizeof(int64_t));
    std::memcpy(clen, S.chunk_len.data(), S.chunk_len.size() * sizeof(int32_t));
    std::memcpy(col, S.col.data(), S.col.size() * sizeof(uint32_t));
    std::memcpy(val, S.val.data(), S.val.size() * sizeof(double));
    return FD_OK;
}

fd_status fd_matrix_export_configs(fd_matrix m, uint64_t *up, uint64_t *dn) {
    if (!m || !up || !dn) return fail(FD_ERR_INVALID, "fd_matrix_export_configs: null argument");
    const std::vector<uint64_t> &cu = m->fmt == FD_FMT_MATFREE ? m->hub.mu : m->cfg_up;
    const std::vector<uint64_t> &cd = m->fmt == FD_FMT_MATFREE ? m->hub.md : m->cfg_dn;
    if (cu.empty()) return fail(FD_ERR_INVALID, "fd_matrix_export_configs: not a Hubbard matrix");
    std::memcpy(up, cu.data(), cu.size() * sizeof(uint64_t));
    std::memcpy(dn, cd.data(), cd.size() * sizeof(uint64_t));
    return FD_OK;
}

void fd_matrix_free(fd_matrix m) {
    if (!m) return;
    free_dev(m->dev);
    delete m;
}

fd_status fd_spmmv(fd_matrix m, fd_dtype dt, int32_t nb, const void *X, int64_t ldx, void *Y, int64_t ldy,
                   void *stream) {
    FD_TRY(need_device(m));
    if (dt != FD_F64 && dt != FD_F32) return fail(FD_ERR_INVALID, "fd_spmmv: bad dtype");
    if (!nb_ok(nb)) return fail(FD_ERR_INVALID, "fd_spmmv: nb must be one of 1, 2, 4, 8, 16, 32, 64");
    FD_TRY(check_block(X, ldx, nb, dt, nb, "fd_spmmv X"));
    FD_TRY(check_block(Y, ldy, nb, dt, nb, "fd_spmmv Y"));
    if (overlap(X, ldx, Y, ldy, m->dev.D, esize(dt))) return fail(FD_ERR_INVALID, "fd_spmmv: X and Y overlap");
    SpmmvCall c;
    c.mode = 0;
    c.nb = nb;
    c.x = X; c.ldx = ldx;
    c.y = Y; c.ldy = ldy;
    return launch_spmmv(m->dev, dt, c, (hipStream_t)stream);
}

fd_status fd_cheb_filter(fd_matrix m, fd_dtype dt, int32_t nb, int32_t nbund, void *V, int64_t ldv,
                         const double *mu, int32_t degree, double alpha, double beta, void *W1, void *W2,
                         int64_t ldw, void *stream) {
    FD_TRY(need_device(m));
    if (dt != FD_F64 && dt != FD_F32) return fail(FD_ERR_INVALID, "fd_cheb_filter: bad dtype");
    if (!nb_ok(nb)) return fail(FD_ERR_INVALID, "fd_cheb_filter: nb must be one of 1, 2, 4, 8, 16, 32, 64");
    if (nbund < 1) return fail(FD_ERR_INVALID, "fd_cheb_filter: n_bundles < 1");
    if (degree < 2) return fail(FD_ERR_INVALID, "fd_cheb_filter: degree must be >= 2");
    if (!mu) return fail(FD_ERR_INVALID, "fd_cheb_filter: null coefficients");
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(FD_ERR_INVALID, "fd_cheb_filter: alpha/beta not finite");
    FD_TRY(check_block(V, ldv, (int64_t)nb * nbund, dt, nb, "fd_cheb_filter V"));
    FD_TRY(check_block(W1, ldw, nb, dt, nb, "fd_cheb_filter W1"));
    FD_TRY(check_block(W2, ldw, nb, dt, nb, "fd_cheb_filter W2"));
    const int64_t D = m->dev.D;
    const size_t es = esize(dt);
    if (overlap(V, ldv, W1, ldw, D, es) || overlap(V, ldv, W2, ldw, D, es) || overlap(W1, ldw, W2, ldw, D, es))
        return fail(FD_ERR_INVALID, "fd_cheb_filter: V, W1, W2 overlap");
    return cheb_filter_impl(m, dt, nb, nbund, V, ldv, mu, degree, alpha, beta, W1, W2, ldw, (hipStream_t)stream);
}

fd_status fd_cheb_coeffs(int32_t kind, double a, double b, int32_t degree, double *mu) {
    return cheb_coeffs(kind, a, b, degree, mu);
}

fd_status fd_gram(int64_t D, int32_t m, int32_t n, const double *X, int64_t ldx, const double *Y, int64_t ldy,
                  double *G, int64_t ldg, void *stream) {
    if (!X || !Y || !G || ldx < m || ldy < n || ldg < n) return fail(FD_ERR_INVALID, "fd_gram: bad arguments");
    return gram(D, m, n, X, ldx, Y, ldy, G, ldg, false, (hipStream_t)stream);
}

fd_status fd_rotate(int64_t D, int32_t m, int32_t n, double *X, int64_t ldx, const double *Q, int64_t ldq,
                    void *stream) {
    if (!X || !Q || ldx < m || ldq < n) return fail(FD_ERR_INVALID, "fd_rotate: bad arguments");
    return rotate(D, m, n, X, ldx, Q, ldq, (hipStream_t)stream);
}

fd_status fd_syev(int32_t n, double *S, int64_t lds, double *w, double *U, int64_t ldu, void *stream) {
    if (!S || !w || !U || lds < n || ldu < n) return fail(FD_ERR_INVALID, "fd_syev: bad arguments");
    return syev(n, S, lds, w, U, ldu, (hipStream_t)stream);
}

int32_t fd_syev_last_sweeps(void) { return last_syev_sweeps(); }

fd_status fd_autotune(fd_matrix m, fd_dtype dt, int32_t nb, int32_t *shape, void *stream) {
    FD_TRY(need_device(m));
    if ((dt != FD_F64 && dt != FD_F32) || !nb_ok(nb)) return fail(FD_ERR_INVALID, "fd_autotune: bad dtype or nb");
    SpmmvTune t;
    FD_TRY(autotune(m->dev, dt, nb, (hipStream_t)stream, &t));
    if (shape) {
        shape[0] = t.order;
        shape[1] = t.xcd;
        shape[2] = t.iters;
        shape[3] = t.grid;
        shape[4] = t.nontemporal;
        shape[5] = t.wide;
        shape[6] = t.tile;
        shape[7] = t.shfl;
        shape[8] = t.lpr;
        shape[9] = t.lds;
    }
    return FD_OK;
}

fd_status kpm_chunk(fd_matrix m, int32_t nb, const double *R, int64_t ldr, int32_t nmom, double alpha,
                    double beta, double *W1, double *W2, int64_t ldw, double *mu, hipStream_t s,
                    double *dots_ws = nullptr, double *part_ws = nullptr);

// Moments over ncol columns in chunks of 64, 32, ... (weighted by width).
// dots_ws / part_ws: device buffers for the moment dots (nmom x 64) and the
// reduction partials (2048 x 64), or nullptr for the process workspace.
fd_status kpm_all(fd_matrix m, int32_t ncol, const double *R, int64_t ldr, int32_t nmom, double alpha, double beta,
                  double *W1, double *W2, int64_t ldw, double *mu, hipStream_t s, double *dots_ws,
                  double *part_ws) {
    FD_TRY(need_device(m));
    if (ncol < 1 || nmom < 2 || (nmom & 1) || !mu) return fail(FD_ERR_INVALID, "fd_kpm_moments: bad ncol or nmom");
    const int wmax = std::min(ncol, 64);
    FD_TRY(check_block(R, ldr, ncol, FD_F64, 1, "fd_kpm_moments R"));
    FD_TRY(check_block(W1, ldw, wmax, FD_F64, 1, "fd_kpm_moments W1"));
    FD_TRY(check_block(W2, ldw, wmax, FD_F64, 1, "fd_kpm_moments W2"));
    const int64_t D = m->dev.D;
    if (overlap_w(W1, ldw, wmax, W2, ldw, wmax, D, 8) || overlap_w(R, ldr, ncol, W1, ldw, wmax, D, 8) ||
        overlap_w(R, ldr, ncol, W2, ldw, wmax, D, 8))
        return fail(FD_ERR_INVALID, "fd_kpm_moments: R, W1, W2 overlap");
    std::vector<double> part(nmom), total(nmom, 0.0);
    // chunks of 64 columns, then the largest power of two that is left
    for (int j = 0; j < ncol;) {
        int w = 64;
        while (w > ncol - j) w >>= 1;
        FD_TRY(kpm_chunk(m, w, R + j, ldr, nmom, alpha, beta, W1, W2, ldw, part.data(), s, dots_ws, part_ws));
        for (int k = 0; k < nmom; k++) total[k] += part[k] * ((double)w / (double)ncol);
        j += w;
    }
    std::copy(total.begin(), total.end(), mu);
    return FD_OK;
}

fd_status fd_kpm_moments(fd_matrix m, int32_t ncol, const double *R, int64_t ldr, int32_t nmom, double alpha,
                         double beta, double *W1, double *W2, int64_t ldw, double *mu, void *stream) {
    return kpm_all(m, ncol, R, ldr, nmom, alpha, beta, W1, W2, ldw, mu, (hipStream_t)stream, nullptr, nullptr);
}

// The moments with the two device buffers carved out of the static scratch
// (no allocation): nmom x 64 doubles of moment dots, then the partial sums
// of the column reductions (at most 2048 x 64 doubles).
fd_status fd_kpm_moments_noalloc(fd_matrix m, int32_t ncol, const double *R, int64_t ldr, int32_t nmom,
                                 double alpha, double beta, double *W1, double *W2, int64_t ldw, double *mu,
                                 void *stream) {
    const size_t need = ((size_t)nmom * 64 + (size_t)2048 * 64) * sizeof(double);
    if (nmom < 2 || nmom > FD_KPM_NOALLOC_MAX_MOMENTS || need > kScratchBytes)
        return fail(FD_ERR_INVALID, "fd_kpm_moments_noalloc: nmom must be even and in [2, 4096]");
    void *base = nullptr;
    FD_TRY(scratch_ptr(&base));
    double *dots = (double *)base, *part = dots + (size_t)nmom * 64;
    return kpm_all(m, ncol, R, ldr, nmom, alpha, beta, W1, W2, ldw, mu, (hipStream_t)stream, dots, part);
}

fd_status fd_kpm_count(const double *mu, int32_t nmom, int32_t damped, int64_t D, double a, double b,
                       double *count) {
    if (!mu || !count || nmom < 1 || D < 0 || (damped != 0 && damped != 1))
        return fail(FD_ERR_INVALID, "fd_kpm_count: bad arguments");
    if (!(mu[0] > 0.0)) return fail(FD_ERR_INVALID, "fd_kpm_count: mu_0 must be positive");
    std::vector<double> c(nmom);
    FD_TRY(cheb_coeffs(damped ? 2 : 0, a, b, nmom - 1, c.data()));
    double n = 0.0;
    for (int k = 0; k < nmom; k++) n += c[k] * mu[k];
    *count = (double)D * n / mu[0];
    return FD_OK;
}

// one chunk of nb <= 64 columns (nb a power of two)
fd_status kpm_chunk(fd_matrix m, int32_t nb, const double *R, int64_t ldr, int32_t nmom, double alpha,
                    double beta, double *W1, double *W2, int64_t ldw, double *mu, hipStream_t stream,
                    double *dots_ws, double *part_ws) {
    // arguments checked by the caller (kpm_all)
    if (!nb_ok(nb)) return fail(FD_ERR_INVALID, "fd_kpm_moments: bad chunk width");
    const int64_t D = m->dev.D;
    hipStream_t s = (hipStream_t)stream;
    const int half = nmom / 2;
    // per column: d[2m] = <T_m|T_m>, d[2m+1] = <T_{m+1}|T_m>, m = 0 .. half-1
    double *dots = dots_ws ? dots_ws : (double *)workspace((size_t)nmom * nb * sizeof(double), 5);
    if (!dots) return fail(FD_ERR_OOM, "fd_kpm_moments: workspace");
    FD_TRY(copy_block(D, nb, R, ldr, W2, ldw, s));  // T_0
    SpmmvCall c;
    c.nb = nb;
    c.mode = 1;  // T_1 = B T_0
    c.x = W2; c.ldx = ldw;
    c.y = W1; c.ldy = ldw;
    c.a = alpha; c.b = beta;
    FD_TRY(launch_spmmv(m->dev, FD_F64, c, s));
    FD_TRY(col_dots(D, nb, W2, ldw, W2, ldw, dots, s, part_ws));
    FD_TRY(col_dots(D, nb, W1, ldw, W2, ldw, dots + nb, s, part_ws));
    double *cur = W1, *prev = W2;  // T_m, T_{m-1}
    for (int k = 1; k < half; k++) {
        c.mode = 4;  // prev <- T_{m+1} = 2 B T_m - T_{m-1}
        c.x = cur; c.ldx = ldw;
        c.z = prev; c.ldz = ldw;
        c.y = prev; c.ldy = ldw;
        c.a = 2.0 * alpha; c.b = 2.0 * beta;
        FD_TRY(launch_spmmv(m->dev, FD_F64, c, s));
        FD_TRY(col_dots(D, nb, cur, ldw, cur, ldw, dots + (size_t)(2 * k) * nb, s, part_ws));
        FD_TRY(col_dots(D, nb, prev, ldw, cur, ldw, dots + (size_t)(2 * k + 1) * nb, s, part_ws));
        std::swap(cur, prev);
    }
    std::vector<double> h((size_t)nmom * nb);
    FD_HIP(hipMemcpyAsync(h.data(), dots, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    FD_HIP(hipStreamSynchronize(s));
    // doubling: T_{2m} = 2 T_m^2 - T_0, T_{2m+1} = 2 T_{m+1} T_m - T_1
    std::vector<double> d(nmom, 0.0);
    for (int k = 0; k < nmom; k++)
        for (int j = 0; j < nb; j++) d[k] += h[(size_t)k * nb + j];
    const double norm = 1.0 / ((double)nb * (double)D);
    mu[0] = d[0] * norm;
    mu[1] = d[1] * norm;
    for (int k = 1; k < half; k++) {
        mu[2 * k] = (2.0 * d[2 * k] - d[0]) * norm;
        mu[2 * k + 1] = (2.0 * d[2 * k + 1] - d[1]) * norm;
    }
    return FD_OK;
}

fd_status fd_pick_degree(fd_matrix m, double tau_lo, double tau_hi, int32_t nt, int32_t ns, const float *params,
                         uint64_t seed, int32_t *degree, double *radius, float *features, void *stream) {
    FD_TRY(need_device(m));
    const double lo = m->lam_lo, hi = m->lam_hi;
    if (!degree || nt < 1 || ns < nt || !(tau_lo <= tau_hi) || tau_lo < lo || tau_hi > hi || !(hi > lo))
        return fail(FD_ERR_INVALID, "fd_pick_degree: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const int64_t D = m->dev.D;
    const int R = 16, M = 256;
    const double alpha = 2.0 / (hi - lo), beta = -(hi + lo) / (hi - lo);
    DevBuf blk;
    FD_TRY(blk.alloc((size_t)D * R * 8 * 3, "KPM blocks"));
    double *Rv = (double *)blk.p, *W1 = Rv + (size_t)D * R, *W2 = W1 + (size_t)D * R;
    FD_TRY(fill_normal(D, R, Rv, R, seed, s));
    std::vector<double> mu(M);
    FD_TRY(fd_kpm_moments(m, R, Rv, R, M, alpha, beta, W1, W2, R, mu.data(), s));
    // counting function D sum_k g_k c_k mu_k: the window coefficients carry
    // the Jackson factors g_k already
    const std::vector<double> &dm = mu;
    const double tau = 0.5 * (tau_lo + tau_hi);
    const double wlo = tau_hi > tau_lo ? tau_lo : lo, whi = tau_hi > tau_lo ? tau_hi : hi;
    const double rt = kpm_radius(dm, D, alpha, beta, tau, wlo, whi, nt);
    const double rs = kpm_radius(dm, D, alpha, beta, tau, lo, hi, ns);
    // Jackson broadening pi (lam_r - lam_l) / (2 (n + 1)) about half the gap
    // between the N_t-th and the N_s-th nearest eigenvalue
    const double gap = std::max(rs - rt, 1e-12 * (hi - lo));
    double n = std::ceil(2.0 * M_PI * (hi - lo) / (2.0 * gap));
    double r = rt;
    if (features || params) {
        std::vector<float> f(FD_MLP_IN);
        std::vector<double> g64(64);  // (2 - delta_k0) g_k T_k(1), Jackson for 64 moments
        FD_TRY(cheb_coeffs(1, 1.0, 0.0, 63, g64.data()));
        for (int k = 0; k < 64; k++) f[k] = (float)(mu[k] * g64[k] / (k == 0 ? 1.0 : 2.0));
        f[64] = (float)(alpha * tau_lo + beta);
        f[65] = (float)(alpha * tau_hi + beta);
        if (features) std::copy(f.begin(), f.end(), features);
        if (params) {
            DevBuf io;
            FD_TRY(io.alloc((FD_MLP_IN + FD_MLP_OUT) * sizeof(float), "picker input"));
            float *xin = (float *)io.p, *yout = xin + FD_MLP_IN;
            FD_HIP(hipMemcpyAsync(xin, f.data(), FD_MLP_IN * sizeof(float), hipMemcpyHostToDevice, s));
            FD_TRY(mlp_forward(params, 1, xin, yout, s));
            float o[FD_MLP_OUT];
            FD_HIP(hipMemcpyAsync(o, yout, sizeof(o), hipMemcpyDeviceToHost, s));
            FD_HIP(hipStreamSynchronize(s));
            if (std::isfinite(o[0]) && std::isfinite(o[1])) {  // else keep the rule
                n *= std::exp2(std::max(-3.0f, std::min(3.0f, o[0])));
                r *= std::exp2(std::max(-3.0f, std::min(3.0f, o[1])));
            }
        }
    }
    *degree = (int32_t)std::max(20.0, std::min(20000.0, n));
    if (radius) *radius = r;
    return FD_OK;
}

fd_status fd_mlp_forward(const float *P, int32_t B, const float *X, float *out, void *stream) {
    return mlp_forward(P, B, X, out, (hipStream_t)stream);
}

fd_status fd_mlp_grad(const float *P, int32_t B, const float *X, const float *Y, const float *w, float *G,
                      float *loss, void *stream) {
    return mlp_grad(P, B, X, Y, w, G, loss, (hipStream_t)stream);
}

fd_status fd_mlp_adam(float *P, const float *G, float *M, float *V, int32_t step, float lr, float wd,
                      void *stream) {
    return mlp_adam(P, G, M, V, step, lr, wd, (hipStream_t)stream);
}

fd_status fd_stream(int32_t op, int64_t n, const double *a, const double *b, double *c, double scalar,
                    void *stream) {
    return stream_op(op, n, a, b, c, scalar, (hipStream_t)stream);
}

fd_status fd_spmmv_tune(int32_t order, int32_t xcd, int32_t iters, int32_t grid, int32_t nontemporal, int32_t wide,
                        int32_t tile, int32_t shfl, int32_t lpr, int32_t lds) {
    if (order < 0 || order > 1 || xcd < 0 || xcd > 2 || (order == 1 && xcd == 2) || iters < 0 || grid < 0 ||
        grid > (1 << 24) || tile < 0 || tile > (1 << 20) || shfl < 0 || shfl > 2 ||
        (lpr != 0 && lpr != 4 && lpr != 8 && lpr != 16) || lds < 0 || lds > 1)
        return fail(FD_ERR_INVALID, "fd_spmmv_tune: bad arguments");
    SpmmvTune &t = spmmv_tune();
    t.order = order;
    t.xcd = xcd;
    t.iters = iters;
    t.grid = grid;
    t.nontemporal = nontemporal != 0;
    t.wide = wide != 0;
    t.tile = tile;
    t.shfl = shfl;
    t.lpr = lpr;
    t.lds = lds;
    return FD_OK;
}

fd_status fd_orthog(int64_t D, int32_t ns, double *V, int64_t ldv, int32_t method, uint64_t seed, int32_t *rank,
                    void *stream) {
    if (!V || D < 1 || ns < 1 || ns > 512 || ldv < ns) return fail(FD_ERR_INVALID, "fd_orthog: bad arguments");
    if (method != FD_ORTHO_SVQB2 && method != FD_ORTHO_CHOLQR2) return fail(FD_ERR_INVALID, "fd_orthog: bad method");
    int r = 0;
    FD_TRY(orthog_impl(D, ns, V, ldv, method, seed, &r, (hipStream_t)stream));
    if (rank) *rank = r;
    return FD_OK;
}

fd_status fd_lehmann(int64_t D, int32_t n, const double *V, const double *W, int64_t ld, double rho,
                     double *lower, int32_t *n_lower, double *upper, int32_t *n_upper, void *stream) {
    if (!V || !W || !lower || !upper || !n_lower || !n_upper || D < 1 || n < 1 || n > 512 || ld < n || n > D ||
        !std::isfinite(rho))
        return fail(FD_ERR_INVALID, "fd_lehmann: bad arguments");
    if (overlap(V, ld, W, ld, D, 8)) return fail(FD_ERR_INVALID, "fd_lehmann: V and W overlap");
    std::vector<double> mu(n);
    FD_TRY(lehmann_impl(D, n, V, W, ld, rho, mu.data(), (hipStream_t)stream));
    // mu ascending: the negative ones give [rho + 1/mu_i, rho) with at least i
    // eigenvalues (i-th most negative first); the positive ones, from the
    // largest, give (rho, rho + 1/mu_i]
    int nl = 0, nu = 0;
    for (int i = 0; i < n; i++)
        if (mu[i] < 0.0) lower[nl++] = rho + 1.0 / mu[i];
    for (int i = n - 1; i >= 0; i--)
        if (mu[i] > 0.0) upper[nu++] = rho + 1.0 / mu[i];
    *n_lower = nl;
    *n_upper = nu;
    return FD_OK;
}

fd_status fd_rayleigh_ritz(fd_matrix m, int32_t ns, int32_t nb, double *V, double *W, int64_t ld, double *theta,
                           double *resid, void *stream) {
    FD_TRY(need_device(m));
    if (!nb_ok(nb) || ns < 1 || ns > 512 || ns % nb) return fail(FD_ERR_INVALID, "fd_rayleigh_ritz: ns must be a multiple of nb <= 512");
    if (!theta || !resid) return fail(FD_ERR_INVALID, "fd_rayleigh_ritz: null output");
    FD_TRY(check_block(V, ld, ns, FD_F64, nb, "fd_rayleigh_ritz V"));
    FD_TRY(check_block(W, ld, ns, FD_F64, nb, "fd_rayleigh_ritz W"));
    if (overlap(V, ld, W, ld, m->dev.D, 8)) return fail(FD_ERR_INVALID, "fd_rayleigh_ritz: V and W overlap");
    return rr_impl(m, ns, nb, V, W, ld, theta, resid, (hipStream_t)stream);
}

fd_status fd_lanczos(fd_matrix m, int32_t k, uint64_t seed, double *theta, double *resid, int32_t *steps,
                     void *stream) {
    FD_TRY(need_device(m));
    if (!theta || !resid || !steps) return fail(FD_ERR_INVALID, "fd_lanczos: null output");
    std::vector<double> th, rs;
    FD_TRY(lanczos_impl(m->dev, 0, k, seed, th, rs, (hipStream_t)stream));
    std::copy(th.begin(), th.end(), theta);
    std::copy(rs.begin(), rs.end(), resid);
    *steps = (int32_t)th.size();
    return FD_OK;
}

fd_status fd_solve(fd_matrix m, const fd_solve_params *P, const double *V0, double *evals, double *evecs,
                   double *resid, fd_solve_stats *stats) {
    FD_TRY(need_device(m));
    if (!P || !evals) return fail(FD_ERR_INVALID, "fd_solve: null argument");
    const int nb = P->nb, ns = P->n_search, nt = P->n_target;
    if (!nb_ok(nb) || ns < nb || ns % nb || ns > 512 || nt < 1 || nt > ns)
        return fail(FD_ERR_INVALID, "fd_solve: need nb in {1..64}, N_s a multiple of nb, N_t <= N_s <= 512");
    if (P->degree < 2 && P->degree != 0) return fail(FD_ERR_INVALID, "fd_solve: degree must be >= 2 (or 0)");
    if (P->max_iter < 0 || !(P->tol > 0)) return fail(FD_ERR_INVALID, "fd_solve: bad max_iter or tol");
    if (P->precision != 0 && P->precision != 1) return fail(FD_ERR_INVALID, "fd_solve: precision must be 0 or 1");
    const double lo = m->lam_lo, hi = m->lam_hi;
    if (!(P->tau_lo <= P->tau_hi) || P->tau_lo < lo || P->tau_hi > hi)
        return fail(FD_ERR_INVALID, "fd_solve: window must satisfy lam_lo <= tau_lo <= tau_hi <= lam_hi");
    if (!(hi > lo)) return fail(FD_ERR_INVALID, "fd_solve: spectrum interval is a point");
    const int64_t D = m->dev.D;
    if (ns > D) return fail(FD_ERR_INVALID, "fd_solve: N_s > D");
    if (P->adapt < 0 || P->adapt > 2) return fail(FD_ERR_INVALID, "fd_solve: adapt must be 0, 1 or 2");
    if (P->interval < 0 || P->interval > 512) return fail(FD_ERR_INVALID, "fd_solve: interval must be in [0, 512]");
    const double t0 = now();
    hipStream_t s = nullptr;
    double normH = 0.0;
    FD_TRY(lanczos_norm(m, normH, s));
    // scaling interval: Gershgorin, or (interval = k > 0) the k-step Lanczos
    // interval widened by the residual bounds and 1 % of its width, inside
    // the Gershgorin one
    double slo = lo, shi = hi;
    if (P->interval > 0) {
        std::vector<double> th, rs;
        FD_TRY(lanczos_impl(m->dev, 0, P->interval, kNormSeed, th, rs, s));
        const double a = th.front() - rs.front(), b = th.back() + rs.back(), w = 0.01 * (b - a);
        slo = std::max(lo, a - w);
        shi = std::min(hi, b + w);
        if (!(shi > slo)) return fail(FD_ERR_BREAKDOWN, "fd_solve: empty Lanczos interval");
    }
    const double alpha = 2.0 / (shi - slo), beta = -(shi + slo) / (shi - slo);
    int degree = P->degree;
    double r0 = -1.0;
    if (degree == 0)
        FD_TRY(fd_pick_degree(m, P->tau_lo, P->tau_hi, nt, ns, P->picker_dev, P->seed ^ 0x5EEDULL, &degree, &r0,
                              nullptr, nullptr));
    std::vector<double> mu(degree + 1);
    // coefficients of the filter for the target window [wlo, whi]
    auto set_coeffs = [&](double wlo, double whi) -> fd_status {
        if (whi > wlo) {
            const double a = std::max(-1.0, std::min(1.0, alpha * wlo + beta));
            const double b = std::max(a, std::min(1.0, alpha * whi + beta));
            return cheb_coeffs(0, a, b, degree, mu.data());
        }
        const double a = std::max(-1.0, std::min(1.0, alpha * wlo + beta));
        return cheb_coeffs(1, a, 0.0, degree, mu.data());
    };
    if (r0 > 0.0 && P->tau_hi > P->tau_lo) {
        const double tau = 0.5 * (P->tau_lo + P->tau_hi);
        FD_TRY(set_coeffs(std::max(P->tau_lo, tau - r0), std::min(P->tau_hi, tau + r0)));
    } else {
        FD_TRY(set_coeffs(P->tau_lo, P->tau_hi));
    }
    // Workspaces: all bundles in one launch when W1/W2 for every bundle fit in
    // 512 MB; otherwise bundle by bundle with nb-wide W1/W2.
    const bool concurrent = (size_t)D * ns * 8 * 2 <= (512ull << 20);
    const int64_t ldw = concurrent ? ns : nb;
    DevBuf V, W, W1, W2, V32;
    FD_TRY(V.alloc((size_t)D * ns * 8, "V"));
    FD_TRY(W.alloc((size_t)D * ns * 8, "W"));
    FD_TRY(W1.alloc((size_t)D * ldw * 8, "W1"));
    FD_TRY(W2.alloc((size_t)D * ldw * 8, "W2"));
    if (P->precision == 1) FD_TRY(V32.alloc((size_t)D * ns * 4, "V32"));
    double *Vd = (double *)V.p, *Wd = (double *)W.p;
    if (V0) {
        FD_HIP(hipMemcpy(Vd, V0, (size_t)D * ns * 8, hipMemcpyHostToDevice));
    } else {
        FD_TRY(fill_normal(D, ns, Vd, ns, P->seed, s));
    }
    // pick the sparse kernels' launch shape for this matrix once (large
    // matrices only: small ones are bound by launch latency)
    if (D >= (1 << 20)) {
        const int di = 0, lg = __builtin_ctz((unsigned)nb);
        if (!m->dev.tuned[di][lg]) FD_TRY(autotune(m->dev, FD_F64, nb, s, nullptr));
        if (P->precision == 1 && !m->dev.tuned[1][lg]) FD_TRY(autotune(m->dev, FD_F32, nb, s, nullptr));
    }
    std::vector<double> th(ns), rho(ns);
    std::vector<int> sel;
    fd_solve_stats st;
    std::memset(&st, 0, sizeof(st));
    st.norm_H = normH;
    st.degree = degree;
    bool fp32 = P->precision == 1;
    // FD_TRACE=1: one JSON line per outer iteration on stderr; FD_TRACE_FILE:
    // the same lines appended to that file (flushed line by line)
    const bool trace = trace_on();
    double prev_max = INFINITY;
    // stagnation: for kStall iterations (FP64 filter) the largest residual
    // of the targets has not dropped below 0.9 of its best value and no more
    // pairs have converged than before (a new target entering the set can
    // hold the largest residual up while the others converge)
    constexpr int kStall = 60;
    double best_max = INFINITY;
    int best_conv = 0;
    int stall = 0;
    bool stagnated = false;
    const double tol = P->tol * normH;
    bool converged = false;
    int it = 0;
    double lehmann_r = INFINITY;
    std::vector<double> lmu(ns);
    for (;;) {
        double ta = now();
        int rank = 0;
        FD_TRY(orthog_impl(D, ns, Vd, ns, P->ortho, P->seed + 0x1000 + it, &rank, s));
        FD_HIP(hipStreamSynchronize(s));
        double tb = now();
        st.t_orthog += tb - ta;
        FD_TRY(rr_impl(m, ns, nb, Vd, Wd, ns, th.data(), rho.data(), s));
        st.t_rr += now() - tb;
        st.spmmv_count += ns / nb;
        for (int j = 0; j < ns; j++)
            if (!std::isfinite(th[j]) || !std::isfinite(rho[j]))
                return fail(FD_ERR_BREAKDOWN, "fd_solve: non-finite Ritz data");
        sel = select_targets(th, P->tau_lo, P->tau_hi, nt);
        // largest residual of the N_t selected pairs (infinite while fewer
        // than N_t Ritz values lie in the window)
        double mx = (int)sel.size() == nt ? 0.0 : INFINITY;
        for (int j : sel) mx = std::max(mx, rho[j]);
        st.n_conv = 0;
        for (int j = 0; j < ns; j++)
            if ((P->tau_hi <= P->tau_lo || (th[j] >= P->tau_lo && th[j] <= P->tau_hi)) && rho[j] <= tol) st.n_conv++;
        converged = (int)sel.size() == nt && mx <= tol;
        const double tau = 0.5 * (P->tau_lo + P->tau_hi);
        if (P->adapt == 2 && P->tau_hi > P->tau_lo && !converged && it < P->max_iter) {
            // certified radius around tau that holds N_t eigenvalues
            const double tl = now();
            fd_status ls = lehmann_impl(D, ns, Vd, Wd, ns, tau, lmu.data(), s);
            lehmann_r = ls == FD_OK ? lehmann_radius(lmu, nt) : INFINITY;
            st.t_rr += now() - tl;
        }
        if (trace) {
            // valid JSON: non-finite values as null
            char mxs[32], lrs[32];
            std::snprintf(mxs, sizeof mxs, std::isfinite(mx) ? "%.3e" : "null", mx / normH);
            std::snprintf(lrs, sizeof lrs, std::isfinite(lehmann_r) ? "%.3e" : "null", lehmann_r);
            char line[512];
            std::snprintf(line, sizeof line,
                          "{\"fd_iter\": %d, \"D\": %lld, \"max_resid_rel\": %s, \"n_in_window\": %d, "
                          "\"n_conv\": %d, \"next_fp32\": %d, \"spmmv\": %lld, \"t_filter\": %.3f, "
                          "\"t_orthog\": %.3f, \"t_rr\": %.3f, \"lehmann_r\": %s, \"t\": %.3f}\n",
                          it, (long long)D, mxs, (int)sel.size(), st.n_conv, (int)fp32, (long long)st.spmmv_count,
                          st.t_filter, st.t_orthog, st.t_rr, lrs, now() - t0);
            trace_line(line);
        }
        if (!fp32) {
            if (mx < 0.9 * best_max || st.n_conv > best_conv) {
                best_max = std::min(best_max, mx);
                best_conv = std::max(best_conv, (int)st.n_conv);
                stall = 0;
            } else {
                stall++;
            }
        }
        stagnated = !converged && stall >= kStall;
        if (converged || it >= P->max_iter || stagnated) break;
        // mixed precision: leave FP32 once the residual is near what an FP32
        // filter can deliver (1e-6 ||H||), or once it stalls (under 10 %
        // progress per iteration) below 1e-3 ||H||
        if (fp32 && std::isfinite(mx) &&
            (mx <= 1e-6 * normH || (mx > 0.9 * prev_max && mx < 1e-3 * normH))) {
            fp32 = false;
            best_max = mx;
            stall = 0;
        }
        prev_max = mx;
        if (P->adapt == 1 && P->tau_hi > P->tau_lo && (int)sel.size() == nt) {
            // target window: tau +- distance of the N_t-th nearest Ritz value
            const double r = std::fabs(th[sel.back()] - tau);
            FD_TRY(set_coeffs(std::max(P->tau_lo, tau - r), std::min(P->tau_hi, tau + r)));
        }
        if (P->adapt == 2 && P->tau_hi > P->tau_lo && std::isfinite(lehmann_r)) {
            // target window: the Lehmann radius, which provably holds N_t
            // eigenvalues (the paper's requirement on the target interval)
            FD_TRY(set_coeffs(std::max(P->tau_lo, tau - lehmann_r), std::min(P->tau_hi, tau + lehmann_r)));
        }
        double tf = now();
        if (fp32) {
            float *V32d = (float *)V32.p;
            FD_TRY(convert_f64_f32(D, ns, Vd, ns, V32d, ns, s));
            FD_TRY(cheb_filter_impl(m, FD_F32, nb, ns / nb, V32d, ns, mu.data(), degree, alpha, beta, W1.p,
                                    W2.p, ldw, s));
            FD_TRY(convert_f32_f64(D, ns, V32d, ns, Vd, ns, s));
            st.iters_fp32++;
        } else {
            FD_TRY(cheb_filter_impl(m, FD_F64, nb, ns / nb, Vd, ns, mu.data(), degree, alpha, beta, W1.p,
                                    W2.p, ldw, s));
        }
        FD_HIP(hipStreamSynchronize(s));
        st.t_filter += now() - tf;
        st.spmmv_count += (int64_t)degree * (ns / nb);
        it++;
    }
    st.iters = it;
    // return the selected pairs sorted by eigenvalue
    std::vector<int> order(sel);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return th[a] < th[b]; });
    const int nret = (int)order.size();
    st.max_resid = 0.0;
    for (int k = 0; k < nt; k++) {
        evals[k] = k < nret ? th[order[k]] : NAN;
        if (resid) resid[k] = k < nret ? rho[order[k]] : NAN;
        if (k < nret) st.max_resid = std::max(st.max_resid, rho[order[k]]);
    }
    if (evecs && nret > 0) {
        int *idx = (int *)workspace(nret * sizeof(int), 4);
        if (!idx) return fail(FD_ERR_OOM, "fd_solve: index workspace");
        FD_HIP(hipMemcpy(idx, order.data(), nret * sizeof(int), hipMemcpyHostToDevice));
        FD_TRY(gather_cols(D, nret, Vd, ns, idx, evecs, nt, s));
        FD_HIP(hipStreamSynchronize(s));
    }
    st.t_total = now() - t0;
    if (stats) *stats = st;
    if (!converged)
        return fail(FD_ERR_NOT_CONVERGED, stagnated ? "fd_solve: stagnated (no 10% progress and no newly converged pair in 60 iterations)"
                                                    : "fd_solve: not converged within max_iter");
    return FD_OK;
}

fd_status fd_debug_alloc_limit(int64_t bytes) {
    if (bytes < 0) return fail(FD_ERR_INVALID, "fd_debug_alloc_limit: bytes must be >= 0");
    g_alloc_limit.store(bytes);
    return FD_OK;
}

// ------------------------------------------------------------- batched FD --
fd_status fd_batch_create(int32_t n_inst, const fd_matrix *mats, fd_batch *out) {
    if (!mats || !out || n_inst < 1 || n_inst > 65535)
        return fail(FD_ERR_INVALID, "fd_batch_create: need 1 <= n_inst <= 65535 and arrays");
    int64_t D = 0, nnz = 0;
    for (int i = 0; i < n_inst; i++) {
        const fd_matrix m = mats[i];
        if (!m) return fail(FD_ERR_INVALID, "fd_batch_create: null matrix");
        if (m->fmt == FD_FMT_MATFREE) return fail(FD_ERR_INVALID, "fd_batch_create: matrix-free matrices have no CSR");
        D += m->csr.D;
        nnz += m->csr.rowptr[m->csr.D];
    }
    if (D >= (int64_t)UINT32_MAX || nnz >= (int64_t)UINT32_MAX)
        return fail(FD_ERR_UNSUPPORTED, "fd_batch_create: more than 2^32 rows or entries in all");
    fd_batch b = new (std::nothrow) fd_batch_s;
    if (!b) return fail(FD_ERR_OOM, "fd_batch_create: host allocation");
    b->off.assign(n_inst + 1, 0);
    std::vector<uint32_t> ptr(D + 1), col(nnz);
    std::vector<double> val(nnz);
    std::vector<uint16_t> inst(D);
    int64_t r = 0, e = 0;
    for (int i = 0; i < n_inst; i++) {
        const HostCSR &A = mats[i]->csr;
        b->lam_lo.push_back(mats[i]->lam_lo);
        b->lam_hi.push_back(mats[i]->lam_hi);
        for (int64_t row = 0; row < A.D; row++) {
            ptr[r + row] = (uint32_t)(e + A.rowptr[row]);
            inst[r + row] = (uint16_t)i;
        }
        const int64_t n = A.rowptr[A.D];
        for (int64_t j = 0; j < n; j++) {
            col[e + j] = (uint32_t)(r + A.col[j]);
            val[e + j] = A.val[j];
        }
        r += A.D;
        e += n;
        b->off[i + 1] = r;
    }
    ptr[D] = (uint32_t)e;
    std::vector<float> v32(val.begin(), val.end());
    BatchDev &d = b->dev;
    d.n_inst = n_inst;
    d.D = D;
    d.minlen = INT32_MAX;
    for (int64_t row = 0; row < D; row++) {
        d.maxlen = std::max<int32_t>(d.maxlen, (int32_t)(ptr[row + 1] - ptr[row]));
        d.minlen = std::min<int32_t>(d.minlen, (int32_t)(ptr[row + 1] - ptr[row]));
    }
    if (d.minlen > d.maxlen) d.minlen = d.maxlen;
    fd_status st = FD_OK;
    auto put = [&](void **dst, const void *src, size_t bytes) {
        if (st != FD_OK) return;
        if (hipMalloc(dst, std::max<size_t>(bytes, 256)) != hipSuccess) {
            *dst = nullptr;
            st = fail(FD_ERR_OOM, "fd_batch_create: device allocation");
            return;
        }
        if (src && bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
            st = fail(FD_ERR_HIP, "fd_batch_create: copy to device");
    };
    put((void **)&d.ptr, ptr.data(), ptr.size() * sizeof(uint32_t));
    put((void **)&d.col, col.data(), col.size() * sizeof(uint32_t));
    put((void **)&d.val64, val.data(), val.size() * sizeof(double));
    put((void **)&d.val32, v32.data(), v32.size() * sizeof(float));
    put((void **)&d.inst, inst.data(), inst.size() * sizeof(uint16_t));
    std::vector<int32_t> ones(n_inst, 1), zeros(n_inst, 0);
    std::vector<double> dz(n_inst, 0.0);
    put((void **)&d.alpha, dz.data(), n_inst * sizeof(double));
    put((void **)&d.beta, dz.data(), n_inst * sizeof(double));
    put((void **)&d.deg, zeros.data(), n_inst * sizeof(int32_t));
    put((void **)&d.act, ones.data(), n_inst * sizeof(int32_t));
    // row structure of the batched dense steps: reduction slices of up to
    // 1024 rows (at most 128 per instance) and 32-row rotation chunks
    std::vector<int32_t> seg_inst, inst_s0(n_inst + 1, 0), rc_inst;
    std::vector<int64_t> seg_r0, seg_r1, rc_r0;
    for (int i = 0; i < n_inst; i++) {
        const int64_t a = b->off[i], Di = b->off[i + 1] - a;
        const int64_t nsl = std::max<int64_t>(1, std::min<int64_t>(128, (Di + 1023) / 1024));
        for (int64_t k = 0; k < nsl; k++) {
            seg_inst.push_back(i);
            seg_r0.push_back(a + k * Di / nsl);
            seg_r1.push_back(a + (k + 1) * Di / nsl);
        }
        inst_s0[i + 1] = (int32_t)seg_inst.size();
        for (int64_t r = a; r < a + Di; r += 32) {
            rc_inst.push_back(i);
            rc_r0.push_back(r);
        }
    }
    if (rc_inst.size() > 0x7fffffff) st = fail(FD_ERR_UNSUPPORTED, "fd_batch_create: too many rows");
    d.nseg = (int32_t)seg_inst.size();
    d.nrc = (int32_t)rc_inst.size();
    put((void **)&d.off, b->off.data(), b->off.size() * sizeof(int64_t));
    put((void **)&d.seg_inst, seg_inst.data(), seg_inst.size() * sizeof(int32_t));
    put((void **)&d.inst_s0, inst_s0.data(), inst_s0.size() * sizeof(int32_t));
    put((void **)&d.seg_r0, seg_r0.data(), seg_r0.size() * sizeof(int64_t));
    put((void **)&d.seg_r1, seg_r1.data(), seg_r1.size() * sizeof(int64_t));
    put((void **)&d.rc_inst, rc_inst.data(), rc_inst.size() * sizeof(int32_t));
    put((void **)&d.rc_r0, rc_r0.data(), rc_r0.size() * sizeof(int64_t));
    if (st == FD_OK && hipGetDevice(&b->device) != hipSuccess) st = fail(FD_ERR_HIP, "fd_batch_create: device");
    if (st != FD_OK) {
        batch_release(b);
        delete b;
        return st;
    }
    *out = b;
    return FD_OK;
}

fd_status fd_batch_info(fd_batch b, int64_t *D_total, int64_t *row_off) {
    if (!b) return fail(FD_ERR_INVALID, "fd_batch_info: null handle");
    if (D_total) *D_total = b->dev.D;
    if (row_off) std::copy(b->off.begin(), b->off.end(), row_off);
    return FD_OK;
}

void fd_batch_free(fd_batch b) {
    if (!b) return;
    batch_release(b);
    delete b;
}

fd_status fd_batch_spmmv(fd_batch b, fd_dtype dt, int32_t nb, const void *X, int64_t ldx, void *Y, int64_t ldy,
                         void *stream) {
    if (!b) return fail(FD_ERR_INVALID, "fd_batch_spmmv: null handle");
    if (dt != FD_F64 && dt != FD_F32) return fail(FD_ERR_INVALID, "fd_batch_spmmv: bad dtype");
    if (!nb_ok(nb)) return fail(FD_ERR_INVALID, "fd_batch_spmmv: nb must be one of 1, 2, 4, 8, 16, 32, 64");
    FD_TRY(check_block(X, ldx, nb, dt, nb, "fd_batch_spmmv X"));
    FD_TRY(check_block(Y, ldy, nb, dt, nb, "fd_batch_spmmv Y"));
    if (overlap(X, ldx, Y, ldy, b->dev.D, esize(dt))) return fail(FD_ERR_INVALID, "fd_batch_spmmv: X and Y overlap");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> ones(b->dev.n_inst, 1);
    FD_TRY(batch_params(b, nullptr, nullptr, nullptr, ones.data(), nullptr, 0, s));
    BatchCall c;
    c.mode = 0;
    c.nb = nb;
    c.x = X; c.ldx = ldx; c.bx = nb;
    c.y = Y; c.ldy = ldy; c.by = nb;
    return launch_batch(b->dev, dt, c, s);
}

fd_status fd_batch_filter(fd_batch b, fd_dtype dt, int32_t nb, int32_t n_bundles, void *V, int64_t ldv,
                          const double *mu, const int32_t *degree, int32_t max_degree, const double *alpha,
                          const double *beta, void *W1, void *W2, int64_t ldw, int32_t use_graph, void *stream) {
    if (!b || !mu || !degree || !alpha || !beta) return fail(FD_ERR_INVALID, "fd_batch_filter: null argument");
    if (dt != FD_F64 && dt != FD_F32) return fail(FD_ERR_INVALID, "fd_batch_filter: bad dtype");
    if (!nb_ok(nb) || n_bundles < 1 || n_bundles > 65535 || max_degree < 2 || max_degree > 100000)
        return fail(FD_ERR_INVALID, "fd_batch_filter: bad nb, n_bundles or max_degree");
    const int n = b->dev.n_inst;
    for (int i = 0; i < n; i++)
        if (degree[i] != 0 && (degree[i] < 2 || degree[i] > max_degree))
            return fail(FD_ERR_INVALID, "fd_batch_filter: degree[i] must be 0 or in [2, max_degree]");
    const int64_t w = (int64_t)nb * n_bundles;
    FD_TRY(check_block(V, ldv, w, dt, nb, "fd_batch_filter V"));
    FD_TRY(check_block(W1, ldw, w, dt, nb, "fd_batch_filter W1"));
    FD_TRY(check_block(W2, ldw, w, dt, nb, "fd_batch_filter W2"));
    const int64_t D = b->dev.D;
    const size_t es = esize(dt);
    if (overlap(V, ldv, W1, ldw, D, es) || overlap(V, ldv, W2, ldw, D, es) || overlap(W1, ldw, W2, ldw, D, es))
        return fail(FD_ERR_INVALID, "fd_batch_filter: V, W1 and W2 must not overlap");
    hipStream_t s = (hipStream_t)stream;
    FD_TRY(batch_params(b, alpha, beta, degree, nullptr, mu, max_degree + 1, s));
    return batch_filter_run(b, dt, nb, n_bundles, (char *)V, ldv, max_degree, (char *)W1, (char *)W2, ldw,
                            use_graph != 0, s);
}

// Launch-shape autotuner of the batched step: the fused Chebyshev step
// (V every other step: k = 3 and k = 4 alternately) timed on scratch blocks
// for XCD chunks of 256 .. 16384 rows and both permute loops; the fastest is
// kept in the handle for (dtype, nb).  nb = 0: also the bundle width among
// 8, 16, 32, 64 that divide ns (all when ns = 0; time per vector; in
// *nb_out).  Overwrites the per-instance
// filter parameters on the device (every filter call sets its own).
static fd_status batch_autotune(fd_batch b, fd_dtype dt, int nb_req, int ns, int *nb_out, int32_t *chunk_out,
                                int32_t *sh_out, hipStream_t s) {
    BatchDev &d = b->dev;
    const int n = d.n_inst;
    const size_t es = esize(dt);
    const int di = dt == FD_F64 ? 0 : 1;
    std::vector<int> nbs;
    if (nb_req == 0) {
        for (int w : {8, 16, 32, 64})
            if (ns == 0 || ns % w == 0) nbs.push_back(w);
        if (nbs.empty()) return fail(FD_ERR_INVALID, "batched autotune: N_s has no bundle width among 8 .. 64");
    } else {
        nbs = {nb_req};
    }
    const int nbmax = *std::max_element(nbs.begin(), nbs.end());
    DevBuf buf;
    FD_TRY(buf.alloc((size_t)d.D * nbmax * es * 3, "batched autotune blocks"));
    FD_HIP(hipMemsetAsync(buf.p, 0, (size_t)d.D * nbmax * es * 3, s));
    std::vector<double> al(n, 0.25), be(n, 0.0), mu((size_t)n * 5, 0.5);
    std::vector<int32_t> dg(n, 4), act(n, 1);
    FD_TRY(batch_params(b, al.data(), be.data(), dg.data(), act.data(), mu.data(), 5, s));
    hipEvent_t e0, e1;
    FD_HIP(hipEventCreate(&e0));
    FD_HIP(hipEventCreate(&e1));
    const int chunks[] = {256, 512, 1024, 2048, 4096, 8192, 16384};
    double best_pv = 1e300;
    int best_nb = nbs[0];
    fd_status st = FD_OK;
    for (int w : nbs) {
        const int lg = __builtin_ctz((unsigned)w);
        const int G = std::max(1, (int)(w * es / 16));  // lanes per row (16 bytes each)
        const int rpb = 256 / std::min(G, 256);
        char *x = (char *)buf.p, *y = x + (size_t)d.D * w * es, *v = y + (size_t)d.D * w * es;
        BatchCall c;
        c.nb = w;
        c.nbundles = 1;
        c.mode = 5;
        c.x = x; c.ldx = w;
        c.z = y; c.ldz = w;
        c.y = y; c.ldy = w;
        c.v = v; c.ldv = w;
        const int reps = (int)std::max<int64_t>(3, std::min<int64_t>(20, (int64_t)4e9 / (int64_t)(d.D * w * es + 1)));
        float best_ms = 1e30f;
        int32_t bc = 1024, bs = 2;
        for (int ch : chunks) {
            if (ch < rpb) continue;
            for (int sh = 1; sh <= 2; sh++) {
                if (sh == 1 && G < 8) continue;  // both loops are the same below 8 lanes
                d.chunk[di][lg] = ch;
                d.sh[di][lg] = (int8_t)sh;
                c.k = 3;
                st = launch_batch(d, dt, c, s);  // warm-up
                if (st != FD_OK) break;
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < reps && st == FD_OK; r++) {
                    c.k = 3 + (r & 1);
                    st = launch_batch(d, dt, c, s);
                }
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (st == FD_OK && ms < best_ms) {
                    best_ms = ms;
                    bc = ch;
                    bs = sh;
                }
            }
            if (st != FD_OK) break;
        }
        if (st != FD_OK) break;
        d.chunk[di][lg] = bc;
        d.sh[di][lg] = (int8_t)bs;
        const double per_vec = best_ms / reps / w;
        if (per_vec < best_pv) {
            best_pv = per_vec;
            best_nb = w;
            if (chunk_out) *chunk_out = bc;
            if (sh_out) *sh_out = bs;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    if (st != FD_OK) return st;
    if (nb_out) *nb_out = best_nb;
    // a captured filter graph holds the old launch shape
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    return FD_OK;
}

fd_status fd_batch_autotune(fd_batch b, fd_dtype dt, int32_t nb, int32_t *shape, void *stream) {
    if (!b) return fail(FD_ERR_INVALID, "fd_batch_autotune: null handle");
    if ((dt != FD_F64 && dt != FD_F32) || (nb != 0 && !nb_ok(nb)) || b->dev.D == 0)
        return fail(FD_ERR_INVALID, "fd_batch_autotune: bad dtype or nb");
    int nbo = nb;
    int32_t ch = 0, sh = 0;
    FD_TRY(batch_autotune(b, dt, nb, 0, &nbo, &ch, &sh, (hipStream_t)stream));
    if (shape) {
        shape[0] = nbo;
        shape[1] = ch;
        shape[2] = sh;
    }
    return FD_OK;
}

fd_status fd_solve_batch(fd_batch b, const fd_solve_params *P, const double *V0, double *evals, double *evecs,
                         double *resid, fd_solve_stats *stats, fd_batch_stats *bstats) {
    if (!b || !P || !evals) return fail(FD_ERR_INVALID, "fd_solve_batch: null argument");
    const int n = b->dev.n_inst;
    int nb = P[0].nb;
    const int ns = P[0].n_search, nt = P[0].n_target, ortho = P[0].ortho;
    if ((nb != 0 && (!nb_ok(nb) || ns < nb || ns % nb)) || ns > 512 || nt < 1 || nt > ns)
        return fail(FD_ERR_INVALID, "fd_solve_batch: need nb in {0, 1..64}, N_s a multiple of nb, N_t <= N_s <= 512");
    for (int i = 0; i < n; i++) {
        const fd_solve_params &p = P[i];
        if (p.nb != P[0].nb || p.n_search != ns || p.n_target != nt || p.ortho != ortho)
            return fail(FD_ERR_INVALID, "fd_solve_batch: nb, N_s, N_t and ortho must agree across instances");
        if (p.precision != 0) return fail(FD_ERR_UNSUPPORTED, "fd_solve_batch: FP64 only (precision 0)");
        if (p.interval != 0) return fail(FD_ERR_UNSUPPORTED, "fd_solve_batch: Gershgorin scaling only (interval 0)");
        if (p.degree < 2 || p.degree > 100000) return fail(FD_ERR_INVALID, "fd_solve_batch: degree must be in [2, 1e5]");
        if (p.max_iter < 0 || !(p.tol > 0) || (p.adapt != 0 && p.adapt != 1))
            return fail(FD_ERR_INVALID, "fd_solve_batch: bad max_iter, tol or adapt");
        if (!(p.tau_lo <= p.tau_hi) || p.tau_lo < b->lam_lo[i] || p.tau_hi > b->lam_hi[i] ||
            !(b->lam_hi[i] > b->lam_lo[i]))
            return fail(FD_ERR_INVALID, "fd_solve_batch: window must satisfy lam_lo <= tau_lo <= tau_hi <= lam_hi");
        if (ns > b->off[i + 1] - b->off[i]) return fail(FD_ERR_INVALID, "fd_solve_batch: N_s > D of an instance");
    }
    const double t0 = now();
    const int64_t D = b->dev.D;
    hipStream_t s = nullptr;
    if (nb == 0) FD_TRY(batch_autotune(b, FD_F64, 0, ns, &nb, nullptr, nullptr, s));
    int max_degree = 0;
    for (int i = 0; i < n; i++) max_degree = std::max(max_degree, P[i].degree);
    const int mstride = max_degree + 1;
    std::vector<double> alpha(n), beta(n), normH(n), mu((size_t)n * mstride, 0.0);
    std::vector<int32_t> deg(n), act(n, 1);
    // coefficients of instance i for the target window [wlo, whi]
    auto set_coeffs = [&](int i, double wlo, double whi) -> fd_status {
        double *m = mu.data() + (size_t)i * mstride;
        const double a = std::max(-1.0, std::min(1.0, alpha[i] * wlo + beta[i]));
        if (whi > wlo) return cheb_coeffs(0, a, std::max(a, std::min(1.0, alpha[i] * whi + beta[i])), P[i].degree, m);
        return cheb_coeffs(1, a, 0.0, P[i].degree, m);
    };
    if (b->lz_norm.empty()) {
        // ||H|| of each instance as in fd_solve: 40 Lanczos steps on the
        // instance's rows of the stacked matrix (its columns carry the
        // instance's first row, so the gathered vector is shifted by it)
        std::vector<double> nrm(n);
        for (int i = 0; i < n; i++) {
            DevMatrix v;
            v.D = b->off[i + 1] - b->off[i];
            v.nslots = v.D;
            v.maxlen = b->dev.maxlen;
            v.ptr = b->dev.ptr + b->off[i];
            v.col = b->dev.col;
            v.val64 = b->dev.val64;
            v.val32 = b->dev.val32;
            std::vector<double> th, rs;
            FD_TRY(lanczos_impl(v, b->off[i], kNormSteps, kNormSeed, th, rs, s));
            nrm[i] = std::max(std::fabs(th.front()), std::fabs(th.back()));
        }
        b->lz_norm = nrm;
    }
    for (int i = 0; i < n; i++) {
        const double lo = b->lam_lo[i], hi = b->lam_hi[i];
        alpha[i] = 2.0 / (hi - lo);
        beta[i] = -(hi + lo) / (hi - lo);
        normH[i] = b->lz_norm[i];
        deg[i] = P[i].degree;
        FD_TRY(set_coeffs(i, P[i].tau_lo, P[i].tau_hi));
    }
    DevBuf V, W, W1, W2;
    FD_TRY(V.alloc((size_t)D * ns * 8, "V"));
    FD_TRY(W.alloc((size_t)D * ns * 8, "W"));
    FD_TRY(W1.alloc((size_t)D * ns * 8, "W1"));
    FD_TRY(W2.alloc((size_t)D * ns * 8, "W2"));
    double *Vd = (double *)V.p, *Wd = (double *)W.p;
    if (V0) {
        FD_HIP(hipMemcpy(Vd, V0, (size_t)D * ns * 8, hipMemcpyHostToDevice));
    } else {
        for (int i = 0; i < n; i++)
            FD_TRY(fill_normal(b->off[i + 1] - b->off[i], ns, Vd + b->off[i] * ns, ns, P[i].seed, s));
    }
    FD_TRY(batch_params(b, alpha.data(), beta.data(), deg.data(), act.data(), mu.data(), mstride, s));
    std::vector<fd_solve_stats> st(n);
    std::vector<std::vector<double>> th(n, std::vector<double>(ns)), rho(n, std::vector<double>(ns));
    std::vector<std::vector<int>> sel(n);
    std::vector<char> conv(n, 0), done(n, 0);
    for (int i = 0; i < n; i++) {
        std::memset(&st[i], 0, sizeof(fd_solve_stats));
        st[i].norm_H = normH[i];
        st[i].degree = P[i].degree;
    }
    fd_batch_stats bs;
    std::memset(&bs, 0, sizeof(bs));
    const int64_t launches0 = b->graph_launches;
    int n_active = n;
    // Dense steps of all instances at once when N_s <= 64 (one launch per
    // step for every instance); larger search spaces go instance by instance.
    const bool dense_b = ns <= 64;
    const size_t nn = (size_t)ns * ns;
    DevBuf Gb, Qb, Ub, Thb, Rhob, Pb, Okb, Mkb;
    std::vector<double> th_all, rho_all;
    std::vector<int32_t> ok_h(n), mk_h(n);
    if (dense_b) {
        FD_TRY(Gb.alloc(n * nn * 8, "batched Gram"));
        FD_TRY(Qb.alloc(n * nn * 8, "batched transforms"));
        FD_TRY(Ub.alloc(n * nn * 8, "batched eigenvectors"));
        FD_TRY(Thb.alloc((size_t)n * ns * 8, "batched Ritz values"));
        FD_TRY(Rhob.alloc((size_t)n * ns * 8, "batched residuals"));
        FD_TRY(Pb.alloc((size_t)b->dev.nseg * nn * 8, "batched partial sums"));
        FD_TRY(Okb.alloc((size_t)n * 4, "batched flags"));
        FD_TRY(Mkb.alloc((size_t)n * 4, "batched mask"));
        th_all.resize((size_t)n * ns);
        rho_all.resize((size_t)n * ns);
    }
    double *Gd = (double *)Gb.p, *Qd = (double *)Qb.p, *Ud = (double *)Ub.p, *Thd = (double *)Thb.p,
           *Rhod = (double *)Rhob.p, *Pd = (double *)Pb.p;
    int32_t *Okd = (int32_t *)Okb.p, *Mkd = (int32_t *)Mkb.p;
    for (int it = 0; n_active > 0; it++) {
        double ta = now();
        if (dense_b && ortho == FD_ORTHO_CHOLQR2) {
            // two Cholesky-QR passes for all active instances; an instance
            // whose Cholesky fails continues alone with SVQB2
            std::vector<char> failed(n, 0);
            for (int pass = 0; pass < 2; pass++) {
                for (int i = 0; i < n; i++) mk_h[i] = !done[i] && !failed[i];
                FD_HIP(hipMemcpy(Mkd, mk_h.data(), n * 4, hipMemcpyHostToDevice));
                FD_TRY(seg_gram(b->dev, ns, Vd, Vd, ns, Mkd, Pd, Gd, s));
                FD_TRY(batched_cholinv(n, ns, Gd, Qd, Okd, Mkd, pass == 1, s));
                FD_HIP(hipMemcpyAsync(ok_h.data(), Okd, n * 4, hipMemcpyDeviceToHost, s));
                FD_HIP(hipStreamSynchronize(s));
                for (int i = 0; i < n; i++)
                    if (mk_h[i] && !ok_h[i]) {
                        failed[i] = 1;
                        mk_h[i] = 0;
                    }
                FD_HIP(hipMemcpy(Mkd, mk_h.data(), n * 4, hipMemcpyHostToDevice));
                FD_TRY(seg_rotate(b->dev, ns, Vd, ns, Qd, Mkd, s));
            }
            for (int i = 0; i < n; i++)
                if (failed[i]) {
                    int rank = 0;
                    FD_TRY(orthog_impl(b->off[i + 1] - b->off[i], ns, Vd + b->off[i] * ns, ns, FD_ORTHO_SVQB2,
                                       P[i].seed + 0x1000 + it, &rank, s));
                }
        } else if (dense_b) {
            // two SVQB passes for all active instances; an instance whose
            // block turns out rank deficient continues alone (SVQB2 with
            // the refill of the clipped directions)
            std::vector<char> failed(n, 0);
            for (int pass = 0; pass < 2; pass++) {
                for (int i = 0; i < n; i++) mk_h[i] = !done[i] && !failed[i];
                FD_HIP(hipMemcpy(Mkd, mk_h.data(), n * 4, hipMemcpyHostToDevice));
                FD_TRY(seg_gram(b->dev, ns, Vd, Vd, ns, Mkd, Pd, Gd, s));
                FD_TRY(batched_svqb(n, ns, Gd, Rhod, Thd, Ud, Qd, Okd, Mkd, s));
                FD_HIP(hipMemcpyAsync(ok_h.data(), Okd, n * 4, hipMemcpyDeviceToHost, s));
                FD_HIP(hipStreamSynchronize(s));
                for (int i = 0; i < n; i++)
                    if (mk_h[i] && ok_h[i] < ns) {
                        failed[i] = 1;
                        mk_h[i] = 0;
                    }
                FD_HIP(hipMemcpy(Mkd, mk_h.data(), n * 4, hipMemcpyHostToDevice));
                FD_TRY(seg_rotate(b->dev, ns, Vd, ns, Qd, Mkd, s));
            }
            for (int i = 0; i < n; i++)
                if (failed[i]) {
                    int rank = 0;
                    FD_TRY(orthog_impl(b->off[i + 1] - b->off[i], ns, Vd + b->off[i] * ns, ns, FD_ORTHO_SVQB2,
                                       P[i].seed + 0x1000 + it, &rank, s));
                }
        } else {
            for (int i = 0; i < n; i++) {
                if (done[i]) continue;
                const int64_t Di = b->off[i + 1] - b->off[i];
                int rank = 0;
                FD_TRY(orthog_impl(Di, ns, Vd + b->off[i] * ns, ns, ortho, P[i].seed + 0x1000 + it, &rank, s));
            }
        }
        FD_HIP(hipStreamSynchronize(s));
        double tb = now();
        bs.t_orthog += tb - ta;
        // W = A V for every active instance in one launch, then the dense
        // Rayleigh-Ritz steps (all instances at once, or one by one)
        BatchCall c;
        c.mode = 0;
        c.nb = nb;
        c.nbundles = ns / nb;
        c.x = Vd; c.ldx = ns; c.bx = nb;
        c.y = Wd; c.ldy = ns; c.by = nb;
        FD_TRY(launch_batch(b->dev, FD_F64, c, s));
        if (dense_b) {
            const int32_t *act = b->dev.act;  // the active instances
            FD_TRY(seg_gram(b->dev, ns, Vd, Wd, ns, act, Pd, Gd, s));
            FD_TRY(batched_sym(n, ns, Gd, s));
            FD_TRY(batched_syev(n, ns, Gd, Thd, Ud, act, s));
            FD_TRY(seg_rotate(b->dev, ns, Vd, ns, Ud, act, s));
            FD_TRY(seg_rotate(b->dev, ns, Wd, ns, Ud, act, s));
            FD_TRY(seg_resid(b->dev, ns, Vd, Wd, ns, Thd, act, Pd, Rhod, s));
            FD_HIP(hipMemcpyAsync(th_all.data(), Thd, (size_t)n * ns * 8, hipMemcpyDeviceToHost, s));
            FD_HIP(hipMemcpyAsync(rho_all.data(), Rhod, (size_t)n * ns * 8, hipMemcpyDeviceToHost, s));
            FD_HIP(hipStreamSynchronize(s));
        }
        n_active = 0;
        for (int i = 0; i < n; i++) {
            if (done[i]) continue;
            const int64_t Di = b->off[i + 1] - b->off[i];
            if (dense_b) {
                std::copy(th_all.begin() + (size_t)i * ns, th_all.begin() + (size_t)(i + 1) * ns, th[i].begin());
                std::copy(rho_all.begin() + (size_t)i * ns, rho_all.begin() + (size_t)(i + 1) * ns, rho[i].begin());
            } else {
                FD_TRY(rr_dense(Di, ns, Vd + b->off[i] * ns, Wd + b->off[i] * ns, ns, th[i].data(), rho[i].data(),
                                s));
            }
            st[i].spmmv_count += ns / nb;
            for (int j = 0; j < ns; j++)
                if (!std::isfinite(th[i][j]) || !std::isfinite(rho[i][j]))
                    return fail(FD_ERR_BREAKDOWN, "fd_solve_batch: non-finite Ritz data");
            const fd_solve_params &p = P[i];
            sel[i] = select_targets(th[i], p.tau_lo, p.tau_hi, nt);
            double mx = (int)sel[i].size() == nt ? 0.0 : INFINITY;
            for (int j : sel[i]) mx = std::max(mx, rho[i][j]);
            const double tol = p.tol * normH[i];
            st[i].n_conv = 0;
            for (int j = 0; j < ns; j++)
                if ((p.tau_hi <= p.tau_lo || (th[i][j] >= p.tau_lo && th[i][j] <= p.tau_hi)) && rho[i][j] <= tol)
                    st[i].n_conv++;
            conv[i] = (int)sel[i].size() == nt && mx <= tol;
            if (conv[i] || st[i].iters >= p.max_iter) {
                done[i] = 1;
                act[i] = 0;
                deg[i] = 0;
                st[i].t_total = now() - t0;
                continue;
            }
            n_active++;
            if (p.adapt == 1 && p.tau_hi > p.tau_lo && (int)sel[i].size() == nt) {
                const double tau = 0.5 * (p.tau_lo + p.tau_hi);
                const double r = std::fabs(th[i][sel[i].back()] - tau);
                FD_TRY(set_coeffs(i, std::max(p.tau_lo, tau - r), std::min(p.tau_hi, tau + r)));
            }
        }
        bs.t_rr += now() - tb;
        if (n_active == 0) break;
        double tf = now();
        FD_TRY(batch_params(b, nullptr, nullptr, deg.data(), act.data(), mu.data(), mstride, s));
        FD_TRY(batch_filter_run(b, FD_F64, nb, ns / nb, (char *)Vd, ns, max_degree, (char *)W1.p, (char *)W2.p,
                                ns, true, s));
        FD_HIP(hipStreamSynchronize(s));
        bs.t_filter += now() - tf;
        for (int i = 0; i < n; i++)
            if (!done[i]) {
                st[i].spmmv_count += (int64_t)P[i].degree * (ns / nb);
                st[i].iters++;
            }
        bs.iters = it + 1;
        if (trace_on()) {
            char line[256];
            std::snprintf(line, sizeof line,
                          "{\"fd_batch_iter\": %d, \"instances\": %d, \"active_after\": %d, \"t_filter\": %.3f, "
                          "\"t_orthog\": %.3f, \"t_rr\": %.3f, \"t\": %.3f}\n",
                          it, n, n_active, bs.t_filter, bs.t_orthog, bs.t_rr, now() - t0);
            trace_line(line);
        }
    }
    // results: selected pairs of each instance sorted by eigenvalue
    bool all = true;
    for (int i = 0; i < n; i++) {
        std::vector<int> order(sel[i]);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return th[i][x] < th[i][y]; });
        const int nret = (int)order.size();
        st[i].max_resid = 0.0;
        for (int k = 0; k < nt; k++) {
            evals[(size_t)i * nt + k] = k < nret ? th[i][order[k]] : NAN;
            if (resid) resid[(size_t)i * nt + k] = k < nret ? rho[i][order[k]] : NAN;
            if (k < nret) st[i].max_resid = std::max(st[i].max_resid, rho[i][order[k]]);
        }
        if (evecs && nret > 0) {
            int *idx = (int *)workspace(nret * sizeof(int), 4);
            if (!idx) return fail(FD_ERR_OOM, "fd_solve_batch: index workspace");
            FD_HIP(hipMemcpy(idx, order.data(), nret * sizeof(int), hipMemcpyHostToDevice));
            FD_TRY(gather_cols(b->off[i + 1] - b->off[i], nret, Vd + b->off[i] * ns, ns, idx,
                               evecs + b->off[i] * nt, nt, s));
            FD_HIP(hipStreamSynchronize(s));
        }
        if (conv[i]) bs.n_converged++;
        all = all && conv[i];
    }
    bs.t_total = now() - t0;
    bs.graph_launches = b->graph_launches - launches0;
    bs.nb = nb;
    if (stats) std::copy(st.begin(), st.end(), stats);
    if (bstats) *bstats = bs;
    if (!all) return fail(FD_ERR_NOT_CONVERGED, "fd_solve_batch: some instances did not converge within max_iter");
    return FD_OK;
}

}  // extern "C"
