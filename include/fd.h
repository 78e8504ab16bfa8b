/*
 * fd.h -- C ABI of libfd, an MI355X (gfx950) implementation of the hot path of
 * filter diagonalization (FD) for sparse symmetric eigenproblems, following
 * Alvermann, Hager & Fehske, "Orthogonal layers of parallelism in large-scale
 * eigenvalue computations" (ACM TOPC; arXiv 2209.01974).
 *
 * The problem (Sec. 1, Sec. 2): a sparse real symmetric matrix A of dimension
 * D; find the N_t eigenpairs nearest a target tau, or inside a target window
 * [tau_l, tau_r], with N_s >= N_t search vectors, to a residual bound
 * rho = ||A v - lambda v||_2.  FD repeats: orthogonalize the search block,
 * one extra SpMV for the Ritz values (Rayleigh-Ritz), convergence test, then
 * the Chebyshev polynomial filter V <- p[A] V (Alg. 1, Alg. 2 captions).
 *
 * Conventions for every call
 *  - Every call returns fd_status; nothing throws across the ABI.  On any
 *    error fd_last_error() returns a message (thread-local, valid until the
 *    next failing call on the same thread).  On FD_ERR_INVALID no output has
 *    been written.
 *  - Dense blocks ("blocks of vectors") are row-major: entry i of vector j of
 *    a block X with leading dimension ldx sits at X[i*ldx + j] (Sec. 3.1 asks
 *    for row-major vector storage).  ld is counted in elements.  Blocks used by
 *    the sparse kernels must be aligned to 16 bytes and ld must be a multiple
 *    of the per-lane vector width (2 for FP64, 4 for FP32, or nb if nb is
 *    smaller); 256-byte alignment is recommended.
 *  - Pointers named *_dev are device pointers (HIP device memory of the
 *    current device); pointers named *_host are host pointers.  Device blocks
 *    are owned by the caller; the library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Kernel-level calls are asynchronous on it; calls that return host data
 *    (fd_rayleigh_ritz, fd_orthog's rank, fd_kpm_moments, fd_pick_degree,
 *    fd_lehmann, fd_solve, fd_solve_batch) and the calls that copy host
 *    parameters first (fd_batch_filter, fd_batch_spmmv) synchronize it.
 *  - The library keeps one device workspace per process for the small dense
 *    steps; calls from several host threads at once are not supported.
 */
#ifndef FD_H
#define FD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FD_OK = 0,
    FD_ERR_INVALID = 1,       /* bad argument; outputs untouched             */
    FD_ERR_OOM = 2,           /* host or device allocation failed            */
    FD_ERR_HIP = 3,           /* a HIP runtime call failed                   */
    FD_ERR_NOT_CONVERGED = 4, /* fd_solve: best pairs written, see stats     */
    FD_ERR_BREAKDOWN = 5,     /* non-finite data or a factorization failed   */
    FD_ERR_UNSUPPORTED = 6    /* valid request outside what is built         */
} fd_status;

typedef enum { FD_F64 = 0, FD_F32 = 1 } fd_dtype;
typedef enum { FD_FMT_CSR = 0, FD_FMT_SELL = 1, FD_FMT_MATFREE = 2, FD_FMT_PENCIL = 3 } fd_format;
typedef enum {
    FD_HUBBARD_RING = 0, /* 1D Hubbard model, L sites, n_up + n_dn fermions  */
    FD_ANDERSON_3D = 1,  /* 3D Anderson lattice, L^3 sites                   */
    FD_DIAGONAL = 2,     /* A = diag(diag[0..n-1])                          */
    FD_USER_CSR = 3      /* caller's CSR (D, rowptr, col, val)              */
} fd_model;

/* Parameters of the generated matrices.
 * FD_HUBBARD_RING: H = -t sum_{<ij>,s} (c+_is c_js + h.c.) + U sum_i n_iu n_id
 *   on L sites (3 <= L <= 62); periodic != 0 closes the ring (fermionic
 *   boundary: the wrap bond carries (-1)^(N_s - 1) for N_s fermions of that
 *   spin).  Basis: spin configurations are L-bit masks with N bits set, ranked
 *   in increasing integer order; row = rank(up) * C(L, n_dn) + rank(down).
 *   The diagonal U * (number of doubly occupied sites) is always stored.
 *   D = C(L, n_up) C(L, n_dn) (the Hubbard dimension of Sec. 4.1).
 *   config_order 1: each species' configurations are labelled in reverse
 *   Cuthill-McKee order of that species' hop graph instead of by rank
 *   (breadth-first from a pseudo-peripheral configuration, neighbours by
 *   increasing hop count, then rank; the visiting order reversed), and row
 *   = label(up) * C(L, n_dn) + label(down).  The matrix is then P A P^T of
 *   the ranked one, entry for entry; configurations one hop apart get
 *   nearby labels, so an up hop's gathered rows lie within a few hundred
 *   slabs of C(L, n_dn) rows.  fd_matrix_export_configs returns the
 *   configuration of every label.  config_order 0 is the ranked basis.
 * FD_ANDERSON_3D: site (x,y,z) -> x + L y + L^2 z, periodic nearest-neighbour
 *   hopping -t, on-site energy W (u_{i+skip} - 1/2), u_k the k-th output
 *   (from 0) of SplitMix64 seeded with `seed` (top 53 bits times 2^-53),
 *   L >= 3, skip >= 0 (draws already used, e.g. for L and W themselves).
 *   tile_x, tile_y (both 0: the numbering above): sites numbered along a
 *   walk of (x, y) tiles of tile_x by tile_y sites instead, tiles in
 *   x-then-y order, each tile over all z (z outermost inside the tile, then
 *   y, then x); row r is the r-th site of the walk.  The matrix is P A P^T
 *   of the naturally numbered one (the same entries, each site keeps its
 *   on-site energy), so its spectrum is the same; a site's lattice
 *   neighbours lie within tile_x * tile_y rows except across tile edges.
 *   Not with FD_FMT_PENCIL (which walks the natural numbering).  L^3 must
 *   stay below 2^31 for the tiled numbering and the pencil walk
 *   (FD_ERR_UNSUPPORTED otherwise).
 * FD_DIAGONAL: n entries from `diag` (host).
 * FD_USER_CSR: D rows, rowptr[D+1] (int64), col (uint32, ascending per row),
 *   val (double); host arrays, copied.  D < 2^32.                          */
typedef struct {
    fd_model model;
    int32_t L, n_up, n_dn, periodic;
    double t, U, W;
    uint64_t seed;
    int64_t n;              /* FD_DIAGONAL */
    const double *diag;     /* FD_DIAGONAL */
    int64_t D;              /* FD_USER_CSR */
    const int64_t *rowptr;  /* FD_USER_CSR */
    const uint32_t *col;    /* FD_USER_CSR */
    const double *val;      /* FD_USER_CSR */
    int64_t skip;           /* FD_ANDERSON_3D */
    int32_t tile_x, tile_y; /* FD_ANDERSON_3D: tiled site numbering (0, 0: natural) */
    int32_t config_order;   /* FD_HUBBARD_RING: 0 ranked, 1 reverse Cuthill-McKee labels */
} fd_model_params;

typedef struct fd_matrix_s *fd_matrix; /* opaque, owned by the library */

#define FD_BUILD_HOST_ONLY 1 /* build host arrays only; no device copy */

/* Build the sparse matrix of the model (Sec. 3.1: A stored row-wise, uint32
 * column indices, S_i = 4).  The canonical form is CSR with ascending columns
 * and the diagonal always stored; FD_FMT_SELL additionally permutes rows into
 * SELL-C-sigma: rows stably sorted by descending length inside windows of
 * sigma rows (perm[new] = old), chunks of C rows (C a power of two, 1..64)
 * stored column-major (entry j of chunk row r at chunk_ptr[c] + j*C + r),
 * padded with value 0 and the row's own index as column; slots past D hold
 * column 0.  Column indices keep the original numbering.  Unless
 * FD_BUILD_HOST_ONLY is set, FP64 values, FP32 values (round to nearest
 * even) and the index arrays are copied to the current device.  The
 * Gershgorin interval of A is computed here.  *out receives a new handle.  */
/* FD_FMT_MATFREE (FD_HUBBARD_RING only): no stored matrix, on the host or
 * the device.  The sparse kernels apply H = H_up x I + I x H_dn + U D from
 * per-species hop tables (the tensor-product structure behind the paper's
 * matrix-free Hubbard SpMV, Sec. 4.2): one pass for the down hops and the
 * diagonal in row order, one for the up hops in tiles of C down-states
 * (C = 0: 16; fd_autotune may choose another tile).  The Gershgorin interval
 * is taken from the tables; fd_matrix_export_csr returns FD_ERR_INVALID;
 * fd_matrix_info reports the hop-table entries as "stored".  sigma is
 * ignored.  C outside [0, 2^20]: FD_ERR_INVALID.                           */
/* FD_FMT_PENCIL (FD_ANDERSON_3D only): the CSR rows, walked by the sparse
 * kernels in pencil order: (x, y) tiles of C by sigma sites (0: 16), each
 * running over all z, tiles in x-then-y order.  A row's z neighbours
 * (L^2 rows away in the natural order) are then a few rows away in the
 * walk.  Stored as SELL-1 with perm[new] = old in that order (see
 * fd_matrix_export_sell); vectors stay in the natural order, and every row
 * is computed exactly as with FD_FMT_CSR.                                  */
fd_status fd_build_matrix(const fd_model_params *params, fd_format fmt, int32_t C,
                          int32_t sigma, int32_t flags, fd_matrix *out);

/* D, stored non-zeros of the CSR form, stored slots of the device format
 * (padding included), and the Gershgorin interval [lam_lo, lam_hi].  Any
 * output pointer may be NULL.                                               */
fd_status fd_matrix_info(fd_matrix m, int64_t *D, int64_t *nnz, int64_t *stored,
                         double *lam_lo, double *lam_hi);

/* Copy the canonical CSR into caller host arrays of D+1, nnz, nnz entries
 * (FD_FMT_MATFREE stores none: FD_ERR_INVALID).                            */
fd_status fd_matrix_export_csr(fd_matrix m, int64_t *rowptr, uint32_t *col, double *val);

/* Copy the SELL-C-sigma arrays (FD_FMT_SELL, or FD_FMT_PENCIL with C = 1)
 * into caller host arrays: perm[D], chunk_ptr[nchunks+1], chunk_len[nchunks],
 * col[stored], val[stored], nchunks = ceil(D / C).  Other formats:
 * FD_ERR_INVALID.                                                           */
fd_status fd_matrix_export_sell(fd_matrix m, int32_t *perm, int64_t *chunk_ptr,
                                int32_t *chunk_len, uint32_t *col, double *val);

/* FD_HUBBARD_RING (any format): the spin configuration (L-bit mask) of
 * every up label into up[C(L, n_up)] and of every down label into
 * dn[C(L, n_dn)], caller host arrays; row a * C(L, n_dn) + b of the matrix is
 * the Fock state (up[a], dn[b]).  Other models: FD_ERR_INVALID.            */
fd_status fd_matrix_export_configs(fd_matrix m, uint64_t *up, uint64_t *dn);

void fd_matrix_free(fd_matrix m);

/* Block SpMV (SpMMV), Sec. 3.1 Eq. SpMVprocess for nb vectors at once:
 * Y = A X, X and Y device blocks D x nb (row-major, ld as above, in dtype).
 * FD_F32 uses the FP32 copy of the values and accumulates in FP32.
 * nb in {1,2,4,8,16,32,64}.  X and Y must not overlap.                     */
fd_status fd_spmmv(fd_matrix m, fd_dtype dtype, int32_t nb, const void *X_dev, int64_t ldx,
                   void *Y_dev, int64_t ldy, void *stream);

/* Chebyshev polynomial filter, Alg. 2 caption: V <- p[B] V with
 * p(x) = sum_{k=0}^{degree} mu[k] T_k(x), B = alpha A + beta, degree >= 2,
 * exactly `degree` SpMMVs per bundle.  V is a D x (nb * n_bundles) device
 * block (ld ldv) filtered bundle by bundle (bundle b = columns
 * [b nb, (b+1) nb)).  W1, W2: device workspaces of D rows, ld ldw.  If
 * ldw >= nb * n_bundles all bundles run in one launch per degree step (each
 * bundle uses its own columns of W1/W2); otherwise the bundles run one after
 * another and W1, W2 need only nb columns.  mu_host holds degree+1 FP64
 * coefficients (rounded to FP32 for FD_F32, as are alpha and beta).       */
fd_status fd_cheb_filter(fd_matrix m, fd_dtype dtype, int32_t nb, int32_t n_bundles,
                         void *V_dev, int64_t ldv, const double *mu_host, int32_t degree,
                         double alpha, double beta, void *W1_dev, void *W2_dev, int64_t ldw,
                         void *stream);

/* Chebyshev coefficients (host, FP64) of the window function, Sec. 2
 * (p(x) = sum_k mu_k T_k(x)): kind 0 = indicator of [a, b] (scaled to
 * [-1, 1]) with Jackson damping for degree+1 moments; kind 1 = Jackson-damped
 * delta at a (b unused); kind 2 = the indicator's plain coefficients (no
 * damping; for moments that carry the damping already).  mu_host has
 * degree+1 entries.                                                         */
fd_status fd_cheb_coeffs(int32_t kind, double a, double b, int32_t degree, double *mu_host);

/* G = X^T Y for device blocks X (D x m, ld ldx) and Y (D x n, ld ldy), FP64,
 * on FP64 MFMA with a fixed-order two-stage reduction over D (bitwise
 * reproducible).  G is a device m x n row-major block (ld ldg).  m, n <= 512.
 * This is the Gram product of SVQB (Sec. 3, stack layout: V^t V).          */
fd_status fd_gram(int64_t D, int32_t m, int32_t n, const double *X_dev, int64_t ldx,
                  const double *Y_dev, int64_t ldy, double *G_dev, int64_t ldg, void *stream);

/* X <- X Q in place, X a device D x m block (ld ldx), Q a device m x n
 * row-major block (ld ldq), n <= m <= 512 (columns n..m-1 of X are left
 * unchanged when n < m).  FP64 MFMA.                                        */
fd_status fd_rotate(int64_t D, int32_t m, int32_t n, double *X_dev, int64_t ldx,
                    const double *Q_dev, int64_t ldq, void *stream);

/* Symmetric eigendecomposition of a small device matrix (n <= 512), FP64,
 * cyclic block Jacobi on the GPU: S = U diag(w) U^t.  S_dev (ld lds) is
 * symmetric; w_dev (n) ascending; U_dev (n x n, ld ldu) eigenvectors in
 * columns.  S_dev is only read.                                            */
fd_status fd_syev(int32_t n, double *S_dev, int64_t lds, double *w_dev, double *U_dev,
                  int64_t ldu, void *stream);

/* Chebyshev moments of the kernel polynomial method (Sec. 4.1 computes the
 * density of states with KPM; Weisse et al. RMP 2006):
 *   mu_k = (1 / (ncol D)) sum_r <r| T_k(alpha A + beta) |r>,  k = 0 .. nmom-1,
 * over the ncol >= 1 columns r of the device block R (D x ncol, ld ldr;
 * random vectors give the stochastic trace).  The columns are taken in
 * chunks of 64 (then 32, 16, ... for the rest), each chunk's average weighted
 * by its width.  nmom even: nmom/2 SpMMVs per chunk with
 * T_2m = 2 T_m^2 - 1 and T_2m+1 = 2 T_m+1 T_m - T_1.  W1, W2: device
 * workspaces of min(ncol, 64) columns (ld ldw).  mu_host: nmom entries.
 * FP64.  Synchronizes.                                                      */
fd_status fd_kpm_moments(fd_matrix m, int32_t ncol, const double *R_dev, int64_t ldr, int32_t nmom,
                         double alpha, double beta, double *W1_dev, double *W2_dev, int64_t ldw,
                         double *mu_host, void *stream);

/* fd_kpm_moments for callers that cannot allocate device memory (code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same moments from the same kernels, with the two device buffers the
 * call needs beyond its arguments -- the per-column moment dots (nmom x 64
 * doubles) and the partial sums of the column reductions (2048 x 64) --
 * placed in a static device array of 4 MiB that the library holds on each
 * device it runs on until the process ends (no hipMalloc or hipFree on any
 * path of this call).  nmom must be even and at most
 * FD_KPM_NOALLOC_MAX_MOMENTS; larger: FD_ERR_INVALID before any work.
 * Every call on one device shares that array and leaves it dirty: calls
 * that overlap on one device (two host threads, or two streams in flight)
 * race and give wrong moments.  Synchronizes, as fd_kpm_moments.           */
#define FD_KPM_NOALLOC_MAX_MOMENTS 4096
fd_status fd_kpm_moments_noalloc(fd_matrix m, int32_t ncol, const double *R_dev, int64_t ldr, int32_t nmom,
                                 double alpha, double beta, double *W1_dev, double *W2_dev, int64_t ldw,
                                 double *mu_host, void *stream);

/* KPM estimate of the number of eigenvalues in the scaled window [a, b]
 * (-1 <= a <= b <= 1) from nmom moments (host): D sum_k c_k mu_k / mu_0 with
 * c_k the window's coefficients (fd_cheb_coeffs kind 0, Jackson-damped for
 * nmom moments, when damped == 0; kind 2, plain, when the moments already
 * carry the damping, damped == 1).  Dividing by mu_0 (1 for an exact trace)
 * removes the norm fluctuation of a stochastic sample.  mu_0 <= 0:
 * FD_ERR_INVALID.                                                           */
fd_status fd_kpm_count(const double *mu_host, int32_t nmom, int32_t damped, int64_t D, double a, double b,
                       double *count);

/* Degree picker network (a refinement of the plain rule): an MLP with FD_MLP_IN
 * inputs (64 Jackson-damped KPM moments of the scaled matrix, then the scaled
 * target window [a, b]), three ReLU layers of FD_MLP_HIDDEN and FD_MLP_OUT
 * outputs (log2 of the degree relative to the KPM rule; log2 of the first
 * filter window's half-width relative to the rule's), FP32.  Parameters: one
 * flat array of FD_MLP_NPARAMS floats, per layer W (out x in, row-major) then
 * b.  All pointers are device pointers; X is B x FD_MLP_IN, outputs B x
 * FD_MLP_OUT, row-major.                                                   */
#define FD_MLP_IN 66
#define FD_MLP_HIDDEN 128
#define FD_MLP_OUT 2
#define FD_MLP_NPARAMS (FD_MLP_HIDDEN * FD_MLP_IN + FD_MLP_HIDDEN + 2 * (FD_MLP_HIDDEN * FD_MLP_HIDDEN + FD_MLP_HIDDEN) + \
                        FD_MLP_OUT * FD_MLP_HIDDEN + FD_MLP_OUT)
fd_status fd_mlp_forward(const float *params_dev, int32_t B, const float *X_dev, float *out_dev, void *stream);
/* Gradient of loss = (1/B) sum_i sum_j w_j (out_ij - Y_ij)^2 with respect to
 * the parameters (G_dev, FD_MLP_NPARAMS floats) and the loss (device float). */
fd_status fd_mlp_grad(const float *params_dev, int32_t B, const float *X_dev, const float *Y_dev,
                      const float *w_dev, float *G_dev, float *loss_dev, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1)
 * with decoupled weight decay wd (p -= lr wd p) on params with gradient G
 * and moment arrays M, V (all FD_MLP_NPARAMS).                             */
fd_status fd_mlp_adam(float *params_dev, const float *G_dev, float *M_dev, float *V_dev, int32_t step,
                      float lr, float wd, void *stream);

/* Filter degree for fd_solve from KPM moments (16 N(0,1) vectors drawn from
 * `seed`, 256 moments): the Jackson-damped counting function gives the
 * radii r_t, r_s around tau = (tau_lo + tau_hi)/2 that hold N_t and N_s
 * eigenvalues; the rule takes the degree whose Jackson broadening
 * pi (lam_r - lam_l) / (2 (n + 1)) is half of r_s - r_t (the search margin of
 * Sec. 2, Fig. 2) and r_t as the first filter window.  With params_dev
 * (degree-picker parameters) the network's two outputs scale the rule's
 * degree and window by 2^out (clamped to 2^[-3, 3]); the rule is the
 * fallback.  degree in [20, 20000].  features_host (FD_MLP_IN floats, may be
 * NULL) receives the network inputs.  Synchronizes.                        */
fd_status fd_pick_degree(fd_matrix m, double tau_lo, double tau_hi, int32_t n_target, int32_t n_search,
                         const float *params_dev, uint64_t seed, int32_t *degree, double *radius,
                         float *features_host, void *stream);

/* Launch-shape autotuner: times the fused Chebyshev steps of this matrix
 * (a step with the V update followed by one without, as the filter
 * alternates them; the better of two passes) for a handful of launch shapes
 * (as in fd_spmmv_tune) on scratch blocks of D x nb (allocated and freed
 * here) and keeps the fastest in the handle for
 * (dtype, nb); later calls on this matrix use it.  shape (10 ints, may be
 * NULL) receives order, xcd, iters, grid, nontemporal, wide, tile, shfl,
 * lpr, lds (lpr > 0: one vector on CSR with lpr lanes per row; lds 1: the
 * matrix-free Hubbard down pass with each slab's column slice in LDS).
 * Synchronizes.                                                            */
fd_status fd_autotune(fd_matrix m, fd_dtype dtype, int32_t nb, int32_t *shape, void *stream);

/* STREAM-style bandwidth kernels on device arrays of n doubles (n even,
 * 16-byte aligned): op 0 copies c = a, op 1 is the triad c = a + scalar b,
 * op 2 only reads a (each thread writes one 16-byte partial sum into c, so
 * n >= 2^19 and c holds at least that many values; a stays unchanged), op 3
 * only writes (c = scalar; a and b unused, may be NULL).  The paper
 * measures its memory bandwidth b_m with STREAM (Sec. 3.2, Eq. EstimateT,
 * Table 4); these give the same figure for the GPU's HBM, and the read-only
 * and write-only passes bound kernels whose traffic is mostly one way.     */
fd_status fd_stream(int32_t op, int64_t n, const double *a_dev, const double *b_dev, double *c_dev,
                    double scalar, void *stream);

/* Outer Jacobi sweeps of the last fd_syev (or internal eigensolve) on this
 * process; a diagnostic for tests and tuning.                               */
int32_t fd_syev_last_sweeps(void);

/* Launch shape of the sparse kernels, process-wide (tuning; results do not
 * depend on it, except lpr below).  order 0: each block walks `iters` consecutive groups of
 * rows (0 = automatic); order 1: grid-stride over `grid` blocks per bundle
 * (0 = automatic).  xcd 1: every XCD owns a contiguous eighth of the rows;
 * xcd 2 (order 0 only): XCD x owns the row chunks x, x+8, x+16, ... of
 * `grid` rows each (0 = 1024).  nontemporal != 0: operands that are streamed
 * once bypass the caches.  wide != 0 (nb >= 16): each lane owns 32 bytes of
 * a row (two 16-byte loads per gathered row) instead of 16.  Matrix-free
 * Hubbard matrices use xcd (1: remap as above, else none), nontemporal,
 * wide, shfl (for their hop tables) and tile (down-states per tile of the
 * up-hop pass, 0: the matrix's default).
 * shfl (entry loop): 0, every lane of a row loads every entry; 1 (at
 * least 4 lanes per row, else as 0), lanes 0..3 of a row load 4 of its
 * entries at once and hand them to the row's other lanes by cross-lane
 * permute; 2 (at least 8 lanes per row, else as 1), the same with lanes
 * 0..7 and 8 entries at once.
 * lpr (one vector, nb = 1, on CSR): 0, a lane owns a row; 4, 8 or 16 lanes
 * share a row, lane q taking its entries q, q + lpr, ... (coalesced index
 * and value loads) and the partial sums added by cross-lane exchanges --
 * the same sum in another order, so results differ by rounding.
 * lds (matrix-free Hubbard): 1 runs the down-hop pass with one block per
 * (up configuration, 16-byte column slice) that first copies the slab's
 * slice into LDS and takes every down hop from there (when the slab's
 * C(L, n_dn) rows of 16 bytes fit in 160 KB and the hops fit the packed
 * 16-bit table; otherwise the plain pass runs); same results bit for bit.
 * Default: order 0, xcd 2, iters 1, grid 1024, nontemporal 1, wide 0,
 * tile 0, shfl 2, lpr 0, lds 0.  A shape chosen by fd_autotune for a matrix takes
 * precedence for that matrix.  tile outside [0, 2^20], shfl outside
 * [0, 2], lpr not in {0, 4, 8, 16} or lds not 0 or 1: FD_ERR_INVALID.        */
fd_status fd_spmmv_tune(int32_t order, int32_t xcd, int32_t iters, int32_t grid, int32_t nontemporal,
                        int32_t wide, int32_t tile, int32_t shfl, int32_t lpr, int32_t lds);

/* Lehmann intervals (Lehmann 1963; Sec. 2 determines the target and search
 * intervals of FD from them).  V_dev: D x n block (ld >= n, linearly
 * independent columns, e.g. the orthonormal search vectors), W_dev = A V
 * (same layout).  For the shift rho the pencil S x = mu B x with
 * S = V^t (A - rho) V and B = ((A - rho) V)^t ((A - rho) V) gives:
 *   lower_host[i] = rho + 1/mu (the i-th most negative mu): [lower[i], rho)
 *     holds at least i+1 eigenvalues of A;          *n_lower such bounds;
 *   upper_host[i] = rho + 1/mu (the i-th largest positive mu): (rho,
 *     upper[i]] holds at least i+1 eigenvalues;     *n_upper such bounds.
 * lower_host and upper_host need n entries each.  All on the GPU (three MFMA
 * Gram products, Cholesky of B, eigenvalues); synchronizes.  B singular
 * (rho an eigenvalue with its eigenvector in span V): FD_ERR_BREAKDOWN.    */
fd_status fd_lehmann(int64_t D, int32_t n, const double *V_dev, const double *W_dev, int64_t ld,
                     double rho, double *lower_host, int32_t *n_lower, double *upper_host,
                     int32_t *n_upper, void *stream);

#define FD_ORTHO_SVQB2 0  /* two SVQB passes (Stathopoulos & Wu 2002)       */
#define FD_ORTHO_CHOLQR2 1 /* two Cholesky-QR passes, SVQB2 if one fails    */

/* Orthonormalize the columns of the device block V (D x ns, ld ldv) in place,
 * FP64 (Sec. 2: orthogonalization after the random start and after each
 * filter; SVQB needs only the ns x ns Gram matrix V^t V).  Columns whose
 * scaled Gram eigenvalue falls below 1e-14 of the largest are replaced by
 * seeded random vectors and orthogonalized again; *rank (may be NULL)
 * receives the number of columns kept.  The second pass of SVQB2 takes
 * (V^t V)^-1/2 from its series when V^t V is within 1e-5 / ns of the
 * identity entrywise (the same span; the basis differs from SVQB's by a
 * rotation).  ns <= 512.  FD_ERR_BREAKDOWN for a non-finite block.
 * Synchronizes stream.                                                    */
fd_status fd_orthog(int64_t D, int32_t ns, double *V_dev, int64_t ldv, int32_t method,
                    uint64_t seed, int32_t *rank, void *stream);

/* Rayleigh-Ritz step (Sec. 2: after each orthogonalization one more SpMMV
 * of the search block gives the Ritz values): W = A V (FP64 SpMMV),
 * H = V^t W, H = Y diag(theta) Y^t,
 * V <- V Y, W <- W Y, rho_j = ||W_j - theta_j V_j||_2.  V must have
 * orthonormal columns.  V, W: device D x ns blocks with the same ld; ns a
 * multiple of nb (nb in {1,...,64}, the bundle width used for A V).
 * theta_host, resid_host: ns entries, theta ascending.  Synchronizes.      */
fd_status fd_rayleigh_ritz(fd_matrix m, int32_t ns, int32_t nb, double *V_dev, double *W_dev,
                           int64_t ld, double *theta_host, double *resid_host, void *stream);

typedef struct {
    double tau_lo, tau_hi; /* target window; tau_lo == tau_hi: nearest tau   */
    int32_t n_target;      /* N_t                                             */
    int32_t n_search;      /* N_s, a multiple of nb, N_t <= N_s <= 512        */
    int32_t nb;            /* bundle width for the filter and SpMMV           */
    int32_t degree;        /* filter degree n >= 2; 0: fd_pick_degree         */
    int32_t max_iter;      /* outer iterations (filter applications)          */
    double tol;            /* converged when rho <= tol * ||H||               */
    int32_t precision;     /* 0: FP64 filter; 1: FP32 filter, FP64 rest       */
    int32_t ortho;         /* FD_ORTHO_SVQB2 or FD_ORTHO_CHOLQR2              */
    uint64_t seed;         /* start block when V0 is NULL                     */
    int32_t adapt;         /* 0: filter for the whole window; 1: each
                              iteration shrink the filter's window around tau
                              to the N_t-th nearest Ritz value in the window
                              (Sec. 2: target interval tracked during FD);
                              2: shrink it to the Lehmann radius at tau, the
                              smallest tau +- r that provably holds N_t
                              eigenvalues (fd_lehmann; Sec. 2)              */
    const float *picker_dev; /* degree 0: degree-picker parameters (device,
                              FD_MLP_NPARAMS) or NULL for the KPM rule     */
    int32_t interval;      /* scaling interval of the filter: 0 Gershgorin;
                              k in [1, 512]: k Lanczos steps (fd_lanczos,
                              seed 1), [theta_1 - r_1, theta_k + r_k] widened
                              by 1 % of its width, inside the Gershgorin
                              interval (Sec. 2: a few steps of Lanczos)    */
} fd_solve_params;

typedef struct {
    int32_t iters;        /* filter applications performed                   */
    int32_t n_conv;       /* Ritz pairs in the window with rho <= tol ||H||   */
    int32_t iters_fp32;   /* of which in FP32 (precision 1)                   */
    int64_t spmmv_count;  /* SpMMVs on nb-vector bundles                      */
    double t_filter, t_orthog, t_rr, t_total; /* seconds                      */
    double norm_H;        /* ||H|| of the test rho <= tol ||H||: the largest
                             |Ritz value| of 40 Lanczos steps (fd_lanczos,
                             seed 1), a lower bound of ||H||_2            */
    double max_resid;     /* largest rho among the returned pairs             */
    int32_t degree;       /* filter degree used                               */
} fd_solve_stats;

/* k steps of Lanczos (Sec. 2: spectral bounds from "a few steps of
 * Lanczos"), FP64, full reorthogonalization (classical Gram-Schmidt against
 * all earlier basis vectors, twice), start vector u_i = 2 U_i - 1 with U_i
 * the i-th output (from 0) of SplitMix64(seed), top 53 bits times 2^-53.
 * Stops early when the new vector's norm drops to 1e-12 of the largest
 * |alpha| (an invariant subspace).  Outputs (caller host arrays of k):
 * theta ascending Ritz values of the tridiagonal, resid their bounds
 * beta_k |s_kj| (each theta_j has an eigenvalue within resid_j); *steps the
 * steps taken (<= min(k, D)).  1 <= k <= 512.  Allocates (k + 1) D doubles
 * of device memory for the basis.  Synchronizes.                           */
fd_status fd_lanczos(fd_matrix m, int32_t k, uint64_t seed, double *theta_host, double *resid_host,
                     int32_t *steps, void *stream);

/* Plain FD (Alg. 1 caption): Gershgorin inclusion interval, alpha and beta,
 * start block V0_host (D x N_s row-major host array) or, if NULL, N(0,1)
 * entries from SplitMix64(seed) by Box-Muller; then repeat orthogonalize ->
 * Rayleigh-Ritz -> convergence test on the N_t Ritz pairs nearest tau inside
 * the window -> filter with the window's Jackson-damped indicator
 * coefficients.  Outputs: evals_host[N_t] ascending, evecs_dev (device
 * D x N_t, ld N_t) or NULL, resid_host[N_t] or NULL, stats or NULL.  Returns
 * FD_ERR_NOT_CONVERGED (outputs written) if max_iter is reached, or
 * earlier once the FP64 filter stagnates: for 60 iterations the largest
 * residual of the targets has not fallen below 0.9 of its best value and
 * the count of converged pairs has not risen above its best.
 * Non-finite data anywhere in the iteration (e.g. NaN in V0_host, or a
 * filter that overflowed) give FD_ERR_BREAKDOWN.  Progress: with the
 * environment variable FD_TRACE=1 fd_solve and fd_solve_batch write one
 * JSON line per outer iteration to stderr; FD_TRACE_FILE=path appends the
 * same lines to that file.                                                 */
fd_status fd_solve(fd_matrix m, const fd_solve_params *params, const double *V0_host,
                   double *evals_host, double *evecs_dev, double *resid_host,
                   fd_solve_stats *stats);

/* ------------------------------------------------------------ batched FD --
 * Many independent problems in one launch per degree step.  The instance
 * matrices are stacked into one block-diagonal CSR on the current device:
 * instance i owns rows [row_off[i], row_off[i+1]) of every batched block
 * and keeps its own inclusion interval, scaling (alpha_i, beta_i), filter
 * coefficients and degree (Alg. 1, Alg. 2 caption, applied per instance).
 * Small problems then share the GPU instead of each being bound by launch
 * latency.  An opaque handle owned by the library.                          */
typedef struct fd_batch_s *fd_batch;

/* Stack n_inst (1..65535) matrices built with a stored format (CSR or SELL;
 * FD_FMT_MATFREE gives FD_ERR_INVALID) into a new batch on the current
 * device.  The matrices stay the caller's and may be freed afterwards.
 * Rows and entries in all < 2^32 (else FD_ERR_UNSUPPORTED).                */
fd_status fd_batch_create(int32_t n_inst, const fd_matrix *mats, fd_batch *out);
/* Total rows D_total and row_off[n_inst + 1] (host, may be NULL).           */
fd_status fd_batch_info(fd_batch b, int64_t *D_total, int64_t *row_off);
void fd_batch_free(fd_batch b);

/* Y = A_i X on the rows of every instance (D_total x nb blocks, as
 * fd_spmmv).  Synchronizes the stream before returning.                    */
fd_status fd_batch_spmmv(fd_batch b, fd_dtype dtype, int32_t nb, const void *X_dev, int64_t ldx,
                         void *Y_dev, int64_t ldy, void *stream);

/* The Chebyshev filter of fd_cheb_filter on every instance at once:
 * V_i <- p_i[alpha_i A_i + beta_i] V_i.  Host arrays: alpha, beta, degree
 * (n_inst each) and mu (n_inst x (max_degree + 1), row i = mu_i0 ..
 * mu_i,max_degree; entries past degree[i] are ignored).  degree[i] = 0
 * leaves instance i untouched, otherwise 2 <= degree[i] <= max_degree
 * <= 100000.  All n_bundles bundles of nb columns run in one launch per
 * degree step: V, W1, W2 are D_total x (nb n_bundles) or wider, pairwise
 * disjoint.  use_graph != 0: the max_degree launches are captured once into
 * a HIP graph kept in the handle (captured again when the buffers, shape or
 * max_degree change) and replayed as one graph launch on `stream`.  The
 * parameters are copied to the device first (the call synchronizes the
 * stream for that); the steps are asynchronous.                            */
fd_status fd_batch_filter(fd_batch b, fd_dtype dtype, int32_t nb, int32_t n_bundles, void *V_dev,
                          int64_t ldv, const double *mu_host, const int32_t *degree_host,
                          int32_t max_degree, const double *alpha_host, const double *beta_host,
                          void *W1_dev, void *W2_dev, int64_t ldw, int32_t use_graph, void *stream);

typedef struct {
    int32_t iters;         /* outer iterations of the batch                  */
    int32_t n_converged;   /* instances whose N_t pairs converged            */
    int64_t graph_launches;/* filter graph replays                           */
    double t_filter, t_orthog, t_rr, t_total; /* seconds, whole batch        */
    int32_t nb;            /* bundle width used (chosen when params nb = 0)  */
} fd_batch_stats;

/* Launch-shape autotuner of the batched kernels: times the fused Chebyshev
 * step on scratch blocks of D_total x nb (allocated and freed here) for XCD
 * chunks of 256 .. 16384 rows and both permute entry loops, and keeps the
 * fastest in the handle for (dtype, nb); nb = 0 also picks the bundle width
 * among 8, 16, 32, 64 by time per vector.  shape (3 ints, may be NULL):
 * nb, chunk rows, entry loop (1: rounds of 4 entries, 2: of 8).  Overwrites
 * the per-instance filter parameters on the device (fd_batch_filter and
 * fd_solve_batch set their own).  Synchronizes.                             */
fd_status fd_batch_autotune(fd_batch b, fd_dtype dtype, int32_t nb, int32_t *shape, void *stream);

/* fd_solve on every instance of the batch (FP64 only: precision must be 0,
 * else FD_ERR_UNSUPPORTED).  params[n_inst]: nb, n_search, n_target and
 * ortho must agree (nb = 0: the library times the batched step and picks
 * the bundle width among 8 .. 64 that divide N_s, and the launch shape,
 * as fd_batch_autotune); the window, degree (2..100000, no picker), max_iter,
 * tol, seed and adapt are per instance.  Each outer iteration
 * orthogonalizes and runs Rayleigh-Ritz (one batched SpMMV for W = A V;
 * with N_s <= 64 every dense step of all instances is one launch, else they
 * go instance by instance; an instance whose Cholesky fails or whose block
 * is rank deficient is orthogonalized alone), drops the instances that
 * converged or reached max_iter, and filters all others with one graph
 * launch.  V0_host
 * (D_total x N_s) or NULL (instance i starts from SplitMix64(seed_i)).
 * Outputs: evals_host[n_inst x N_t] (row i ascending), evecs_dev
 * (D_total x N_t, ld N_t) or NULL, resid_host[n_inst x N_t] or NULL,
 * stats[n_inst] or NULL (t_total = time from the start of the batch to the
 * instance's last Rayleigh-Ritz; t_filter/t_orthog/t_rr are 0 there and
 * batch-wide in bstats), bstats or NULL.  FD_ERR_NOT_CONVERGED (outputs
 * written) if any instance reached max_iter.                               */
fd_status fd_solve_batch(fd_batch b, const fd_solve_params *params, const double *V0_host,
                         double *evals_host, double *evecs_dev, double *resid_host,
                         fd_solve_stats *stats, fd_batch_stats *bstats);

/* Test hook for the out-of-memory path: while bytes > 0, every device
 * buffer that fd_solve, fd_solve_batch or fd_lanczos would allocate above
 * that size fails with FD_ERR_OOM (nothing is allocated); 0 lifts the limit.
 * Process-wide.  bytes < 0: FD_ERR_INVALID.                                 */
fd_status fd_debug_alloc_limit(int64_t bytes);

const char *fd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FD_H */
