// Internal declarations shared by the libfd translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fd.h"

namespace fd {

// ------------------------------------------------------------------ errors --
fd_status fail(fd_status st, const std::string &msg);
fd_status hip_fail(hipError_t e, const char *what);

#define FD_HIP(call)                                                      \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) return ::fd::hip_fail(e_, #call);           \
    } while (0)

#define FD_TRY(call)                                                      \
    do {                                                                  \
        fd_status s_ = (call);                                            \
        if (s_ != FD_OK) return s_;                                       \
    } while (0)

// ------------------------------------------------------------ host matrix --
struct HostCSR {
    int64_t D = 0;
    std::vector<int64_t> rowptr;
    std::vector<uint32_t> col;
    std::vector<double> val;
};

struct HostSELL {
    int32_t C = 1, sigma = 1;
    std::vector<int32_t> perm;       // perm[new] = old
    std::vector<int64_t> chunk_ptr;  // nchunks + 1
    std::vector<int32_t> chunk_len;  // nchunks
    std::vector<uint32_t> col;
    std::vector<double> val;
};

// order 0: spin configurations labelled by rank; 1: breadth-first labels of
// each species' hop graph (reverse Cuthill-McKee).  cfg_up / cfg_dn receive
// the configuration (bit mask) of each label; row (a, b) = a n_dn + b.
fd_status build_hubbard(int L, int nup, int ndn, bool periodic, double t, double U, int order, HostCSR &A,
                        std::vector<uint64_t> &cfg_up, std::vector<uint64_t> &cfg_dn);

// Tensor-product form of the Hubbard ring: H = H_up x I + I x H_dn + U D.
// Per spin species, the configurations one hop away (rank, element), sorted.
struct HubbardTables {
    int64_t nu = 0, nd = 0;
    double U = 0;
    std::vector<uint64_t> mu, md;           // spin configurations (bit masks)
    std::vector<int32_t> off_u, off_d;      // nu + 1, nd + 1
    std::vector<int32_t> idx_u, idx_d;      // hop targets (ranks)
    std::vector<double> val_u, val_d;       // hop elements
};
fd_status hubbard_tables(int L, int nup, int ndn, bool periodic, double t, double U, int order, HubbardTables &T);
int64_t hubbard_tables_nnz(const HubbardTables &T);  // non-zeros of the full matrix
void hubbard_tables_gershgorin(const HubbardTables &T, double &lo, double &hi);
fd_status build_anderson(int L, double t, double W, uint64_t seed, int64_t skip, HostCSR &A);
fd_status build_diagonal(int64_t n, const double *d, HostCSR &A);
fd_status build_user(int64_t D, const int64_t *rowptr, const uint32_t *col, const double *val,
                     HostCSR &A);
fd_status build_sell(const HostCSR &A, int C, int sigma, HostSELL &S);
fd_status fill_sell(const HostCSR &A, HostSELL &S);  // chunks from S.C and S.perm
fd_status build_pencil(const HostCSR &A, int L, int tx, int ty, HostSELL &S);
fd_status relabel_tiles(int L, int tx, int ty, HostCSR &A);  // sites numbered along the tile walk
void gershgorin(const HostCSR &A, double &lo, double &hi);
fd_status cheb_coeffs(int kind, double a, double b, int n, double *mu);

// --------------------------------------------------------- device matrix --
// Defaults from sweeps on MI355X (Anderson L=200, nb 1..64, FP64/FP32): one
// row group per block keeps the rows in flight in one compact window, so the
// far neighbours of the gather (+-L^2) are still in the Infinity Cache; the
// blocks are spread over the 8 XCDs in chunks of 1024 consecutive rows, so
// that near neighbours (+-1, +-L) are in the same XCD's L2.  Contiguous
// per-XCD eighths (8 windows) overflowed the Infinity Cache at nb = 64.
struct SpmmvTune {
    int order = 0;        // 0: consecutive row groups per block; 1: grid-stride
    int xcd = 2;          // 1: contiguous eighth per XCD; 2: interleaved row chunks
    int iters = 1;        // order 0: row groups per block (0: automatic)
    int grid = 1024;      // order 1: blocks per bundle; xcd 2: rows per chunk
    int nontemporal = 1;  // 1: streamed operands bypass the caches
    int wide = 0;         // 1: 32 bytes per lane (nb >= 16)
    int tile = 0;         // matrix-free Hubbard: down-state tile of the up pass (0: 16)
    int shfl = 2;         // entry loop: 0 plain; 1 permute rounds of 4 (>= 4 lanes per row); 2 of 8 (>= 8)
    int lpr = 0;          // nb = 1 on CSR: lanes that share a row (4, 8, 16; 0: one lane per row)
    int lds = 0;          // matrix-free Hubbard: 1 stages each slab's column slice in LDS for the down pass
};

// One layout serves CSR and SELL: "slot" s of the device format belongs to
// chunk s >> cshift; its entries start at ptr[chunk] + (s & (C-1)) and step
// by C; the chunk length is (ptr[chunk+1] - ptr[chunk]) >> cshift.  CSR is
// the case C = 1 (cshift 0, ptr = rowptr) with no permutation.
struct DevMatrix {
    int64_t D = 0;
    int32_t cshift = 0;
    int64_t nslots = 0;        // D rounded up to a multiple of C
    int32_t maxlen = 0;        // longest row (C = 1) or chunk
    int32_t minlen = 0;        // shortest row (C = 1) or chunk
    int64_t stored = 0;        // value slots incl. padding
    uint32_t *ptr = nullptr;   // nchunks + 1
    uint32_t *col = nullptr;   // stored
    double *val64 = nullptr;   // stored
    float *val32 = nullptr;    // stored
    int32_t *perm = nullptr;   // nslots (SELL) or null (CSR); -1 for padding slots
    // launch shapes chosen by fd_autotune, per dtype and log2(nb)
    bool tuned[2][7] = {};
    SpmmvTune tune[2][7];
    // matrix-free Hubbard (format FD_FMT_MATFREE): device copies of the tables
    bool matfree = false;
    int64_t nu = 0, nd = 0;
    double U = 0;
    uint64_t *mu = nullptr, *md = nullptr;
    int32_t *off_u = nullptr, *off_d = nullptr, *idx_u = nullptr, *idx_d = nullptr;
    double *val_u64 = nullptr, *val_d64 = nullptr;
    float *val_u32 = nullptr, *val_d32 = nullptr;
    int32_t mf_tile = 16;  // default down-state tile of the up pass
    int32_t mf_maxu = 0, mf_maxd = 0;  // most hops of an up / down state
    uint16_t *hop16_d = nullptr;  // down hops packed (target | 0x8000 for +tmag_d), or null
    double tmag_d = 0;            // |element| shared by every down hop
};

}  // namespace fd

struct fd_matrix_s {
    fd_format fmt = FD_FMT_CSR;
    fd::HostCSR csr;
    fd::HostSELL sell;
    fd::HubbardTables hub;
    std::vector<uint64_t> cfg_up, cfg_dn;  // Hubbard: spin configuration of each label
    int64_t D = 0, nnz = 0, stored = 0;
    double lam_lo = 0, lam_hi = 0;
    double lz_norm = -1.0;  // ||H|| estimate of the convergence test (lazily, by Lanczos)
    int device = -1;
    fd::DevMatrix dev;
};

namespace fd {

// -------------------------------------------------------- kernel launchers --
// Sparse kernels (fd_spmmv.hip).  mode: 0 y = A x; 1 y = a A x + b x;
// 2 t = a A x + b x - v, y = t, v = cv v + cx x + ct t;
// 3 t = a A x + b x - z, y = t (y may alias z), v = v + ct t;
// 4 t = a A x + b x - z, y = t (y may alias z).
struct SpmmvCall {
    int mode = 0;
    int nb = 1;
    int nbundles = 1;          // bundles in this launch (grid y)
    const void *x = nullptr;   int64_t ldx = 0; int64_t bx = 0;  // bx: column offset per bundle
    void *y = nullptr;         int64_t ldy = 0; int64_t by = 0;
    const void *z = nullptr;   int64_t ldz = 0; int64_t bz = 0;
    void *v = nullptr;         int64_t ldv = 0; int64_t bv = 0;
    double a = 1, b = 0, cv = 0, cx = 0, ct = 0;
};
fd_status launch_spmmv(const DevMatrix &M, fd_dtype dt, const SpmmvCall &c, hipStream_t s);
// matrix-free Hubbard form of the same call (fd_hubbard_mf.hip)
fd_status launch_spmmv_mf(const DevMatrix &M, fd_dtype dt, const SpmmvCall &c, const SpmmvTune &tn,
                          hipStream_t s);

SpmmvTune &spmmv_tune();
fd_status autotune(DevMatrix &M, fd_dtype dt, int nb, hipStream_t s, SpmmvTune *best);

// Batched problems (fd_batch.hip): n_inst independent matrices stacked as one
// block-diagonal CSR; instance i owns rows [off[i], off[i+1]).  Per-instance
// scaling, filter coefficients and degree live in device arrays, so one
// launch per degree step serves every instance and bundle.
struct BatchDev {
    int32_t n_inst = 0;
    int64_t D = 0;
    uint32_t *ptr = nullptr, *col = nullptr;  // D + 1, nnz (columns already shifted)
    int32_t maxlen = 0;                       // longest row
    int32_t minlen = 0;                       // shortest row
    // launch shape per dtype and log2(nb) (fd_batch_autotune): rows per XCD
    // chunk (a power of two, 0: 1024) and the entry loop (1: permute rounds
    // of 4 entries, 2: of 8 with 8 or more lanes per row)
    int32_t chunk[2][7] = {};
    int8_t sh[2][7] = {{2, 2, 2, 2, 2, 2, 2}, {2, 2, 2, 2, 2, 2, 2}};
    double *val64 = nullptr;
    float *val32 = nullptr;
    uint16_t *inst = nullptr;  // row -> instance
    double *alpha = nullptr, *beta = nullptr;  // n_inst
    int32_t *deg = nullptr;  // n_inst: rows of instance i take part in steps k <= deg[i]
    int32_t *act = nullptr;  // n_inst: rows take part in the plain SpMMV when act[i] != 0
    double *mu = nullptr;    // n_inst x mstride filter coefficients
    int32_t mstride = 0;
    // row structure for the batched dense steps: instance row offsets, the
    // slices of the Gram / residual reductions (slice s of instance i: rows
    // [seg_r0[s], seg_r1[s]), slices of i: [inst_s0[i], inst_s0[i+1])) and
    // the 32-row chunks of the rotations
    int64_t *off = nullptr;
    int32_t nseg = 0, nrc = 0;
    int32_t *seg_inst = nullptr, *inst_s0 = nullptr, *rc_inst = nullptr;
    int64_t *seg_r0 = nullptr, *seg_r1 = nullptr, *rc_r0 = nullptr;
};
// Batched dense steps (fd_batch_dense.hip), n <= 64 columns per instance.
fd_status seg_gram(const BatchDev &B, int n, const double *X, const double *Y, int64_t ld, const int32_t *mask,
                   double *P, double *G, hipStream_t s);
fd_status seg_rotate(const BatchDev &B, int n, double *X, int64_t ld, const double *Q, const int32_t *mask,
                     hipStream_t s);
fd_status seg_resid(const BatchDev &B, int n, const double *V, const double *W, int64_t ld, const double *theta,
                    const int32_t *mask, double *P, double *rho, hipStream_t s);
fd_status batched_sym(int n_inst, int n, double *G, hipStream_t s);
// as cholqr_transform, one matrix per instance (mask[i] = 0: skipped)
fd_status batched_cholinv(int n_inst, int n, double *G, double *Q, int32_t *ok, const int32_t *mask,
                          bool second_pass, hipStream_t s);
fd_status batched_syev(int n_inst, int n, const double *S, double *w, double *U, const int32_t *mask, hipStream_t s);
// SVQB transform Q of each instance from its Gram matrix G (overwritten);
// rank[i]: directions above the clipping floor.  d: n_inst x n, lam: n_inst x n.
fd_status batched_svqb(int n_inst, int n, double *G, double *d, double *lam, double *U, double *Q, int32_t *rank,
                       const int32_t *mask, hipStream_t s);
struct BatchCall {
    int mode = 0;  // 0: y = A x; 1: first step; 2: second step; 3: step k >= 3
    int k = 0;
    int nb = 1, nbundles = 1;
    const void *x = nullptr;
    int64_t ldx = 0, bx = 0;
    void *y = nullptr;
    int64_t ldy = 0, by = 0;
    const void *z = nullptr;
    int64_t ldz = 0, bz = 0;
    void *v = nullptr;
    int64_t ldv = 0, bv = 0;
};
fd_status launch_batch(const BatchDev &B, fd_dtype dt, const BatchCall &c, hipStream_t s);

// Dense kernels (fd_dense.hip).
fd_status gram(int64_t D, int m, int n, const double *X, int64_t ldx, const double *Y,
               int64_t ldy, double *G, int64_t ldg, bool sym, hipStream_t s);
fd_status rotate(int64_t D, int m, int n, double *X, int64_t ldx, const double *Q, int64_t ldq,
                 hipStream_t s);
fd_status syev(int n, double *S, int64_t lds, double *w, double *U, int64_t ldu, hipStream_t s);
int last_syev_sweeps();
fd_status col_resid(int64_t D, int n, const double *V, const double *W, int64_t ld,
                    const double *theta, double *rho, hipStream_t s);
// SVQB transform: Q = Dg U L^-1/2 from Gram G (n x n, dense ld n); returns
// the rank in *rank_dev (device int) and a keep-mask (device int[n]).
fd_status svqb_transform(int n, double *G, double *Q, double *work, int *keep, int *rank_dev,
                         hipStream_t s);
// CholQR transform Q = R^-1 from the Gram matrix (overwritten); *ok_dev = 0
// on a relative pivot below 1e-14 n, or (second_pass) when G is not within
// 0.5 of the identity entrywise.
fd_status cholqr_transform(int n, double *G, double *Q, int *ok_dev, bool second_pass, hipStream_t s);
// Symmetric second pass Q = G^-1/2 = I - E/2 + 3 E^2 / 8 for G = I + E
// (E, E2: n x n scratch); *ok_dev = 0 and Q untouched when n max|E_ij| > 1e-5.
fd_status lowdin_transform(int n, const double *G, double *E, double *E2, double *Q, int *ok_dev, hipStream_t s);
fd_status refill_random(int64_t D, int n, double *V, int64_t ldv, const int *keep,
                        uint64_t seed, hipStream_t s);
fd_status fill_normal(int64_t D, int n, double *V, int64_t ldv, uint64_t seed, hipStream_t s);
fd_status convert_f64_f32(int64_t D, int n, const double *src, int64_t lds, float *dst,
                          int64_t ldd, hipStream_t s);
fd_status convert_f32_f64(int64_t D, int n, const float *src, int64_t lds, double *dst,
                          int64_t ldd, hipStream_t s);
fd_status gather_cols(int64_t D, int n, const double *src, int64_t lds, const int *idx,
                      double *dst, int64_t ldd, hipStream_t s);
fd_status symmetrize(int n, double *H, hipStream_t s);
// Lehmann pencil (B, S) from the three Gram matrices of V and W = A V
fd_status lehmann_pencil(int n, const double *G2, const double *G1, const double *G0, double rho, double *B,
                         double *S, hipStream_t s);
// out[off + j] = sum_i A[i][j] B[i][j] for j < n (two-stage, fixed order);
// P: the partial sums (at most 2048 n doubles) or nullptr for the workspace
fd_status col_dots(int64_t D, int n, const double *A, int64_t lda, const double *B, int64_t ldb, double *out,
                   hipStream_t s, double *P = nullptr);
// The static device scratch of the entry points that do not allocate:
// kScratchBytes per device, its address on the current device in *out.
constexpr size_t kScratchBytes = 4u << 20;
fd_status scratch_ptr(void **out);
fd_status copy_block(int64_t D, int n, const double *src, int64_t lds, double *dst, int64_t ldd, hipStream_t s);
fd_status copy_rows(int64_t D, int64_t row_bytes, const void *src, int64_t src_ld_bytes, void *dst,
                    int64_t dst_ld_bytes, hipStream_t s);
fd_status stream_op(int op, int64_t n, const double *a, const double *b, double *c, double sc, hipStream_t s);
// Lanczos building blocks; the basis vectors lie one after another (vector t
// at Q + t D).  c[t] = Q_t . w for t < n (two-stage, nblk partial sums in P,
// fixed summation order); w -= sum_t c[t] Q_t; w *= f; q = the seeded start
// vector (2 U_i - 1, U_i the i-th uniform of SplitMix64(seed)).
fd_status lz_dots(int64_t D, int n, const double *Q, const double *w, double *c, double *P, int nblk,
                  hipStream_t s);
fd_status lz_sub(int64_t D, int n, const double *Q, const double *c, double *w, hipStream_t s);
fd_status lz_scale(int64_t D, double *w, double f, hipStream_t s);
fd_status lz_start(int64_t D, double *q, uint64_t seed, hipStream_t s);

// Degree-picker network (fd_mlp.hip).
fd_status mlp_forward(const float *P, int B, const float *X, float *out, hipStream_t s);
fd_status mlp_grad(const float *P, int B, const float *X, const float *Y, const float *wj, float *G,
                   float *loss_dev, hipStream_t s);
fd_status mlp_adam(float *P, const float *G, float *M, float *V, int step, float lr, float wd, hipStream_t s);

// Process-wide device workspace for the small dense steps.
void *workspace(size_t bytes, int slot);

}  // namespace fd
