// Sparse kernels for gfx950: block SpMV (SpMMV) and the fused Chebyshev step.
//
// Sec. 3.1 (Eq. SpMVprocess, Eq. traffic): y_i = sum_j A_ij x_j for n_b
// vectors at once, vectors row-major so that one row of the block (n_b
// values) is contiguous; each matrix entry is loaded once per n_b vectors.
// Alg. 2 caption: the SpMV and the vector updates of the Chebyshev step are
// one kernel, so that W2 is not reloaded (kappa = 5 in Sec. 3.2, Eq. EstimateT).
//
// Mapping on a 64-wide wavefront: a row of the block (nb values) is split
// over G lanes that each own VEC consecutive values (16-byte loads when the
// row is wide enough); a wave covers 64/G rows at a time, a 256-thread block
// 256/G rows, and each block walks `iters` such row groups.  The first 4
// or 8 lanes of a row load that many of its entries (column, value) at once
// and pass them to the row's other lanes by cross-lane permute (with fewer
// lanes per row, every lane loads every entry as a broadcast); the gathered
// rows x[col] are read with one 16-byte load per lane.  With SELL-C-sigma the C rows of a chunk
// read entry j from consecutive addresses (coalesced); CSR is SELL-1-1.
// The rows in flight form one compact window (small blocks in launch order)
// so that the gathered neighbours of a row are found in L2 / Infinity Cache;
// the streamed operands (y, v, z) use non-temporal loads and stores.  A
// per-XCD row partition and a grid-stride order are available as tunables.
#include <type_traits>
#include <vector>

#include "fd_internal.h"

namespace fd {
namespace {

template <typename T, int VEC> struct VecT;
template <> struct VecT<double, 1> { typedef double type; };
template <> struct VecT<double, 2> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct VecT<float, 1> { typedef float type; };
template <> struct VecT<float, 2> { typedef float __attribute__((ext_vector_type(2))) type; };
template <> struct VecT<float, 4> { typedef float __attribute__((ext_vector_type(4))) type; };
template <> struct VecT<double, 4> { typedef double __attribute__((ext_vector_type(4))) type; };
template <> struct VecT<float, 8> { typedef float __attribute__((ext_vector_type(8))) type; };

template <typename T>
struct KArgs {
    const uint32_t *__restrict__ ptr;
    const uint32_t *__restrict__ col;
    const T *__restrict__ val;
    const int32_t *__restrict__ perm;
    int64_t nslots;
    int64_t ngroups;   // row groups of 256/G slots
    int64_t nblk;      // logical blocks (order 0)
    int32_t cshift;
    int32_t iters;
    int32_t xcd;
    int32_t order;     // 0: a block walks `iters` consecutive groups; 1: grid-stride
    int32_t sg;        // xcd == 2: logical blocks per super-group
    int32_t maxlen;    // longest row (CSR) or chunk (SELL)
    int32_t uniform;   // every row (chunk) holds maxlen entries
    const T *x; int64_t ldx, bx;
    T *y; int64_t ldy, by;
    const T *z; int64_t ldz, bz;
    T *v; int64_t ldv, bv;
    T a, b, cv, cx, ct;
};

template <typename V>
__device__ __forceinline__ V ld(const void *p) { return *reinterpret_cast<const V *>(p); }
template <typename V>
__device__ __forceinline__ void st(void *p, V x) { *reinterpret_cast<V *>(p) = x; }
// streamed operands (read or written once per step): non-temporal, so that
// they do not evict the gathered rows of x from L2 / Infinity Cache
// acc + a x with one rounding per element (an explicit FMA, so that every
// variant of the entry loop rounds the same way)
template <typename V, typename T>
__device__ __forceinline__ V fmav(T a, V x, V acc) { return __builtin_elementwise_fma((V)a, x, acc); }
template <typename V, bool NT>
__device__ __forceinline__ V lds(const void *p) {
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    else return *reinterpret_cast<const V *>(p);
}
template <typename V, bool NT>
__device__ __forceinline__ void sts(void *p, V x) {
    if constexpr (NT) __builtin_nontemporal_store(x, reinterpret_cast<V *>(p));
    else *reinterpret_cast<V *>(p) = x;
}

// Row groups of this block.  order 0: groups [b iters, (b+1) iters) of
// logical block b; order 1: grid-stride, so that the blocks running at a
// time cover one compact window of rows.  With xcd != 0 the hardware's
// round-robin of workgroups over the 8 XCDs is undone: XCD x owns the
// x-th eighth of the groups.  g1 <= g0 when the block has no work.
template <typename T>
__device__ __forceinline__ void block_groups(const KArgs<T> &p, int64_t &g0, int64_t &g1, int64_t &gstep) {
    if (p.order == 0) {
        int64_t blk = blockIdx.x;
        if (p.xcd == 1) {
            const int64_t per = (p.nblk + 7) >> 3;
            blk = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
        } else if (p.xcd == 2) {
            // XCD x owns super-groups x, x + 8, x + 16, ... of sg blocks each:
            // one compact window of rows overall, neighbouring rows on one XCD
            const int64_t j = blockIdx.x >> 3;
            blk = ((j / p.sg) * 8 + (blockIdx.x & 7)) * p.sg + (j % p.sg);
        }
        gstep = 1;
        if (blk >= p.nblk) {
            g0 = g1 = 0;
            return;
        }
        g0 = blk * p.iters;
        g1 = min(p.ngroups, g0 + p.iters);
    } else if (p.xcd) {
        const int64_t per = (p.ngroups + 7) >> 3;
        const int64_t x = blockIdx.x & 7;
        g0 = x * per + (blockIdx.x >> 3);
        g1 = min(p.ngroups, (x + 1) * per);
        gstep = gridDim.x >> 3;
    } else {
        g0 = blockIdx.x;
        g1 = p.ngroups;
        gstep = gridDim.x;
    }
}

// UNI: every row (chunk) holds p.maxlen entries (no wave exchange needed)
template <typename T, int VEC, int G, int MODE, bool PERM, bool NT, int SH, bool UNI>
__global__ __launch_bounds__(256) void k_spmmv(KArgs<T> p) {
    typedef typename VecT<T, VEC>::type V;
    constexpr int RPB = 256 / G;
    int64_t g0, g1, gstep;
    block_groups(p, g0, g1, gstep);
    const int64_t bnd = blockIdx.y;
    const T *x = p.x + bnd * p.bx;
    T *y = p.y + bnd * p.by;
    const int grp = threadIdx.x / G;
    const int q = threadIdx.x % G;
    const uint32_t step = 1u << p.cshift;
    for (int64_t g = g0; g < g1; g += gstep) {
        const int64_t s = g * RPB + grp;
        uint32_t len, base, wlen;
        int64_t row;
        V zi = (V)0, vi = (V)0;
        T *vr = nullptr;
        if constexpr (SH == 0 || UNI) {
            // no exchange between the rows of the wave (broadcast loop, or
            // rows of one length: the permute rounds run to maxlen), so a
            // lane may leave at once
            if (s >= p.nslots) break;
            const int64_t c = s >> p.cshift;
            const uint32_t p0 = p.ptr[c];
            len = (p.ptr[c + 1] - p0) >> p.cshift;
            base = p0 + (uint32_t)(s & (step - 1));
            row = PERM ? (int64_t)p.perm[s] : s;
            if (row < 0) continue;  // padding slot past D
            wlen = (uint32_t)p.maxlen;
            // streamed operands first: their latency overlaps the gather chain
            if constexpr (MODE >= 2) {
                vr = p.v + bnd * p.bv + row * p.ldv + q * VEC;
                if constexpr (MODE >= 3) zi = lds<V, NT>(p.z + bnd * p.bz + row * p.ldz + q * VEC);
                if constexpr (MODE == 2 || MODE == 3 || MODE == 5) vi = lds<V, NT>(vr);
            }
        } else {
            // every lane of the block reaches this point (the loop bounds
            // are per block), so the wave can agree on its longest row
            const bool in = s < p.nslots;
            len = 0;
            base = 0;
            row = -1;
            if (in) {
                const int64_t c = s >> p.cshift;
                const uint32_t p0 = p.ptr[c];
                len = (p.ptr[c + 1] - p0) >> p.cshift;
                base = p0 + (uint32_t)(s & (step - 1));
                row = PERM ? (int64_t)p.perm[s] : s;
                // streamed operands first: their latency overlaps the
                // exchange below and the gather chain
                if (row >= 0) {
                    if constexpr (MODE >= 2) {
                        vr = p.v + bnd * p.bv + row * p.ldv + q * VEC;
                        if constexpr (MODE >= 3) zi = lds<V, NT>(p.z + bnd * p.bz + row * p.ldz + q * VEC);
                        if constexpr (MODE == 2 || MODE == 3 || MODE == 5) vi = lds<V, NT>(vr);
                    }
                }
            }
            if (row < 0) len = 0;
            // load rounds of the permute loop: the longest row of this wave
            // (lanes of a row share len, so only the rows are compared)
            wlen = len;
#pragma unroll
            for (int o = G; o < 64; o <<= 1) wlen = max(wlen, (uint32_t)__shfl_xor((int)wlen, o, 64));
            // the same value in every lane: make it a scalar, so that the
            // round loop below is a scalar loop
            wlen = (uint32_t)__builtin_amdgcn_readfirstlane((int)min(wlen, (uint32_t)p.maxlen));
            if (!in) break;
            if (row < 0) continue;  // padding slot past D
        }
        const T *xq = x + q * VEC;
        // the row's own x (the beta term): loaded with the streams, so that
        // its latency is not added after the gathers
        V xi = (V)0;
        if constexpr (MODE != 0) xi = ld<V>(xq + row * p.ldx);
        V acc0 = (V)0, acc1 = (V)0;
        if constexpr (SH != 0) {
            // Entries in load rounds of LW: lanes 0..LW-1 of the row load one
            // entry each (one load instruction for the indices, one for the
            // values, instead of one broadcast load per entry), the other
            // lanes of the row take them by cross-lane permute, 4 at a time,
            // and the gathers go out together (the compiler issues all LW
            // gathers of a round before their FMAs).  The rounds run to the
            // longest row of the wave, so every lane of a row takes part in
            // every permute.
            constexpr int LW = SH == 2 ? 8 : 4;
            constexpr int GW = 4;
            static_assert(G >= LW, "a load round needs LW lanes per row");
            const int rbase = (int)(threadIdx.x & 63) - q;
            for (int j0 = 0; j0 < (int)wlen; j0 += LW) {
                const uint32_t jj = (uint32_t)(j0 + q);
                uint32_t cm = 0;
                T am = (T)0;
                if (q < LW && jj < len) {
                    const uint32_t k = base + jj * step;
                    cm = p.col[k];
                    am = p.val[k];
                }
#pragma unroll
                for (int r0 = 0; r0 < LW; r0 += GW) {
                    uint32_t cc[GW];
                    T aa[GW];
#pragma unroll
                    for (int u = 0; u < GW; u++) {
                        cc[u] = (uint32_t)__shfl((int)cm, rbase + r0 + u, 64);
                        aa[u] = __shfl(am, rbase + r0 + u, 64);
                    }
                    V xs[GW];
#pragma unroll
                    for (int u = 0; u < GW; u++)
                        xs[u] = ((uint32_t)(j0 + r0 + u) < len) ? ld<V>(xq + (int64_t)cc[u] * p.ldx) : (V)0;
                    // even entries to acc0, odd ones to acc1, as in the plain loop
#pragma unroll
                    for (int u = 0; u < GW; u++)
                        if ((uint32_t)(j0 + r0 + u) < len) {
                            if ((r0 + u) & 1) acc1 = fmav(aa[u], xs[u], acc1);
                            else acc0 = fmav(aa[u], xs[u], acc0);
                        }
                }
            }
        } else {
        uint32_t j = 0;
        for (; j + 4 <= len; j += 4) {
            const uint32_t k = base + j * step;
            const uint32_t c0 = p.col[k], c1 = p.col[k + step];
            const uint32_t c2 = p.col[k + 2 * step], c3 = p.col[k + 3 * step];
            const T a0 = p.val[k], a1 = p.val[k + step];
            const T a2 = p.val[k + 2 * step], a3 = p.val[k + 3 * step];
            const V x0 = ld<V>(xq + (int64_t)c0 * p.ldx);
            const V x1 = ld<V>(xq + (int64_t)c1 * p.ldx);
            const V x2 = ld<V>(xq + (int64_t)c2 * p.ldx);
            const V x3 = ld<V>(xq + (int64_t)c3 * p.ldx);
            acc0 = fmav(a0, x0, acc0);
            acc1 = fmav(a1, x1, acc1);
            acc0 = fmav(a2, x2, acc0);
            acc1 = fmav(a3, x3, acc1);
        }
        // at most three entries left (j is a multiple of 4): even, odd, even
        if (j < len) acc0 = fmav(p.val[base + j * step], ld<V>(xq + (int64_t)p.col[base + j * step] * p.ldx), acc0);
        if (j + 1 < len)
            acc1 = fmav(p.val[base + (j + 1) * step], ld<V>(xq + (int64_t)p.col[base + (j + 1) * step] * p.ldx), acc1);
        if (j + 2 < len)
            acc0 = fmav(p.val[base + (j + 2) * step], ld<V>(xq + (int64_t)p.col[base + (j + 2) * step] * p.ldx), acc0);
        }
        const V acc = acc0 + acc1;
        T *yr = y + row * p.ldy + q * VEC;
        if constexpr (MODE == 0) {
            sts<V, NT>(yr, acc);
        } else {
            V t = p.a * acc + p.b * xi;
            if constexpr (MODE == 1) {
                sts<V, NT>(yr, t);
            } else if constexpr (MODE == 2) {
                t -= vi;
                sts<V, NT>(yr, t);
                sts<V, NT>(vr, p.cv * vi + p.cx * xi + p.ct * t);
            } else if constexpr (MODE == 3) {
                t -= zi;
                sts<V, NT>(yr, t);
                sts<V, NT>(vr, vi + p.ct * t);
            } else if constexpr (MODE == 5) {
                // two accumulation terms at once: the previous step's vector
                // (x, whose own row is loaded anyway) and this step's
                t -= zi;
                sts<V, NT>(yr, t);
                sts<V, NT>(vr, vi + p.cx * xi + p.ct * t);
            } else {  // MODE 4: recurrence only (odd filter steps, KPM moments)
                t -= zi;
                sts<V, NT>(yr, t);
            }
        }
    }
}

// One vector (nb = 1), CSR: LPR lanes share a row.  Lane q takes entries
// q, q + LPR, ... of the row, so the row's column indices and values are
// read by consecutive lanes (coalesced), and the LPR partial sums are
// added by a butterfly of cross-lane exchanges; the row's first lane then
// applies the step's update.  (With one lane per row, every lane reads its
// own row's entries, scattered across memory.)
template <typename T, int LPR, int MODE, bool NT>
__global__ __launch_bounds__(256) void k_spmv_vec(KArgs<T> p) {
    constexpr int RPB = 256 / LPR;
    int64_t g0, g1, gstep;
    block_groups(p, g0, g1, gstep);
    const int64_t bnd = blockIdx.y;
    const T *x = p.x + bnd * p.bx;
    T *y = p.y + bnd * p.by;
    const int grp = threadIdx.x / LPR;
    const int q = threadIdx.x % LPR;
    for (int64_t g = g0; g < g1; g += gstep) {
        const int64_t s = g * RPB + grp;
        // every lane of the block reaches the exchanges below (the loop
        // bounds are per block); lanes of a row share s
        const bool in = s < p.nslots;
        T acc = (T)0;
        if (in) {
            const uint32_t k1 = p.ptr[s + 1];
            for (uint32_t k = p.ptr[s] + q; k < k1; k += LPR) acc = fma(p.val[k], x[(int64_t)p.col[k] * p.ldx], acc);
        }
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (!in) break;
        if (q != 0) continue;
        const int64_t row = s;
        T *yr = y + row * p.ldy;
        if constexpr (MODE == 0) {
            sts<T, NT>(yr, acc);
        } else {
            const T xi = x[row * p.ldx];
            T t = p.a * acc + p.b * xi;
            if constexpr (MODE == 1) {
                sts<T, NT>(yr, t);
            } else {
                T *vr = p.v + bnd * p.bv + row * p.ldv;
                if constexpr (MODE == 2) {
                    const T vi = lds<T, NT>(vr);
                    t -= vi;
                    sts<T, NT>(yr, t);
                    sts<T, NT>(vr, p.cv * vi + p.cx * xi + p.ct * t);
                } else {
                    t -= lds<T, NT>(p.z + bnd * p.bz + row * p.ldz);
                    sts<T, NT>(yr, t);
                    if constexpr (MODE == 3) sts<T, NT>(vr, lds<T, NT>(vr) + p.ct * t);
                    if constexpr (MODE == 5) sts<T, NT>(vr, lds<T, NT>(vr) + p.cx * xi + p.ct * t);
                }
            }
        }
    }
}

template <typename T, int VEC, int G, bool VROW = false>
fd_status launch_t(const DevMatrix &M, const T *val, const SpmmvCall &c, hipStream_t s) {
    KArgs<T> p;
    p.ptr = M.ptr;
    p.col = M.col;
    p.val = val;
    p.perm = M.perm;
    p.nslots = M.nslots;
    p.cshift = M.cshift;
    p.maxlen = M.maxlen;
    p.uniform = M.minlen == M.maxlen ? 1 : 0;
    constexpr int RPB = 256 / G;
    const int lg = __builtin_ctz((unsigned)c.nb);
    const int di = std::is_same<T, double>::value ? 0 : 1;
    const SpmmvTune &tn = M.tuned[di][lg] ? M.tune[di][lg] : spmmv_tune();
    p.ngroups = (M.nslots + RPB - 1) / RPB;
    p.order = tn.order;
    p.xcd = tn.xcd;
    int64_t gx;
    if (p.order == 0) {
        int iters = tn.iters;
        if (iters <= 0) {
            // about 8192 blocks or more per bundle for a large matrix
            int64_t want = M.nslots / ((int64_t)RPB * 8192);
            iters = (int)std::max<int64_t>(1, std::min<int64_t>(64, want));
        }
        p.iters = iters;
        p.nblk = (p.ngroups + iters - 1) / iters;
        p.sg = 1;
        if (p.xcd == 2) {
            const int64_t rows = tn.grid > 0 ? tn.grid : 1024;  // super-group size in rows
            p.sg = (int32_t)std::max<int64_t>(1, rows / ((int64_t)RPB * iters));
            const int64_t q = 8LL * p.sg;
            gx = (p.nblk + q - 1) / q * q;
        } else {
            gx = p.xcd ? ((p.nblk + 7) / 8) * 8 : p.nblk;
        }
    } else {
        p.iters = 0;
        p.nblk = 0;
        p.sg = 1;
        int64_t want = tn.grid > 0 ? tn.grid : 2048;
        gx = std::min<int64_t>(want, std::max<int64_t>(8, p.ngroups));
        gx = (gx + 7) / 8 * 8;
    }
    p.x = (const T *)c.x; p.ldx = c.ldx; p.bx = c.bx;
    p.y = (T *)c.y; p.ldy = c.ldy; p.by = c.by;
    p.z = (const T *)c.z; p.ldz = c.ldz; p.bz = c.bz;
    p.v = (T *)c.v; p.ldv = c.ldv; p.bv = c.bv;
    p.a = (T)c.a; p.b = (T)c.b; p.cv = (T)c.cv; p.cx = (T)c.cx; p.ct = (T)c.ct;
    if (gx > 0x7fffffff) return fail(FD_ERR_UNSUPPORTED, "SpMMV: grid too large");
    dim3 grid((unsigned)gx, (unsigned)c.nbundles), block(256);
    const bool perm = M.perm != nullptr;
    const bool nt = tn.nontemporal != 0;
    if constexpr (VROW) {
        if (perm || M.cshift != 0) return fail(FD_ERR_INVALID, "SpMMV: the lane-shared row loop needs CSR");
#define FD_V(MODE)                                                                                  \
    do {                                                                                            \
        if (nt) hipLaunchKernelGGL((k_spmv_vec<T, G, MODE, true>), grid, block, 0, s, p);           \
        else hipLaunchKernelGGL((k_spmv_vec<T, G, MODE, false>), grid, block, 0, s, p);             \
    } while (0)
        switch (c.mode) {
            case 0: FD_V(0); break;
            case 1: FD_V(1); break;
            case 2: FD_V(2); break;
            case 3: FD_V(3); break;
            case 4: FD_V(4); break;
            case 5: FD_V(5); break;
            default: return fail(FD_ERR_INVALID, "SpMMV: bad mode");
        }
#undef FD_V
        FD_HIP(hipGetLastError());
        return FD_OK;
    }
    // entry loop: 0 plain, 1 permute rounds of 4 entries, 2 load rounds of 8;
    // each form needs its lanes per row, else the next smaller one is used
    const int sh = (tn.shfl >= 2 && G >= 8) ? 2 : (tn.shfl != 0 && G >= 4 ? 1 : 0);
    constexpr int S1 = G >= 4 ? 1 : 0, S2 = G >= 8 ? 2 : S1;
    const bool uni = p.uniform != 0;
#define FD_L(MODE, PERM, NT)                                                                                  \
    do {                                                                                                      \
        if (sh == 2 && uni) hipLaunchKernelGGL((k_spmmv<T, VEC, G, MODE, PERM, NT, S2, true>), grid, block, 0, s, p); \
        else if (sh == 2) hipLaunchKernelGGL((k_spmmv<T, VEC, G, MODE, PERM, NT, S2, false>), grid, block, 0, s, p); \
        else if (sh == 1 && uni) hipLaunchKernelGGL((k_spmmv<T, VEC, G, MODE, PERM, NT, S1, true>), grid, block, 0, s, p); \
        else if (sh == 1) hipLaunchKernelGGL((k_spmmv<T, VEC, G, MODE, PERM, NT, S1, false>), grid, block, 0, s, p); \
        else hipLaunchKernelGGL((k_spmmv<T, VEC, G, MODE, PERM, NT, 0, false>), grid, block, 0, s, p);              \
    } while (0)
#define FD_L2(MODE, PERM) \
    if (nt) FD_L(MODE, PERM, true); else FD_L(MODE, PERM, false)
    switch (c.mode * 2 + (perm ? 1 : 0)) {
        case 0: FD_L2(0, false); break;
        case 1: FD_L2(0, true); break;
        case 2: FD_L2(1, false); break;
        case 3: FD_L2(1, true); break;
        case 4: FD_L2(2, false); break;
        case 5: FD_L2(2, true); break;
        case 6: FD_L2(3, false); break;
        case 7: FD_L2(3, true); break;
        case 8: FD_L2(4, false); break;
        case 9: FD_L2(4, true); break;
        case 10: FD_L2(5, false); break;
        case 11: FD_L2(5, true); break;
        default: return fail(FD_ERR_INVALID, "SpMMV: bad mode");
    }
#undef FD_L2
#undef FD_L
    FD_HIP(hipGetLastError());
    return FD_OK;
}

}  // namespace

SpmmvTune &spmmv_tune() {
    static SpmmvTune t;
    return t;
}

// Launch-shape autotuner: time the fused Chebyshev step (the kernel the
// filter repeats) for a few shapes on scratch blocks and keep the fastest
// for this matrix, dtype and nb.
fd_status autotune(DevMatrix &M, fd_dtype dt, int nb, hipStream_t s, SpmmvTune *best_out) {
    const size_t es = dt == FD_F64 ? 8 : 4;
    const size_t bytes = (size_t)M.D * nb * es;
    void *buf = nullptr;
    FD_HIP(hipMalloc(&buf, 3 * bytes));
    FD_HIP(hipMemsetAsync(buf, 0, 3 * bytes, s));
    hipEvent_t e0, e1;
    FD_HIP(hipEventCreate(&e0));
    FD_HIP(hipEventCreate(&e1));
    // order, xcd, iters, grid, nontemporal, wide, tile, shfl
    const SpmmvTune cands[] = {
        {0, 2, 1, 256, 1, 0, 0, 2},  {0, 2, 1, 512, 1, 0, 0, 2},  {0, 2, 1, 1024, 1, 0, 0, 2},
        {0, 2, 1, 2048, 1, 0, 0, 2}, {0, 2, 1, 8192, 1, 0, 0, 2}, {0, 2, 2, 2048, 1, 0, 0, 2},
        {0, 0, 1, 0, 1, 0, 0, 2},    {0, 1, 1, 0, 1, 0, 0, 2},    {1, 1, 1, 4096, 1, 0, 0, 2},
        {0, 2, 1, 512, 1, 0, 0, 1},  {0, 2, 1, 1024, 1, 0, 0, 1}, {0, 2, 1, 2048, 1, 0, 0, 1},
        {0, 2, 1, 8192, 1, 0, 0, 1}, {0, 2, 1, 1024, 1, 1, 0, 0}, {0, 2, 1, 4096, 1, 1, 0, 0},
        {0, 2, 1, 2048, 1, 0, 0, 0}, {0, 2, 1, 8192, 1, 0, 0, 0},
        // one vector on CSR: 4, 8 or 16 lanes per row
        {0, 2, 1, 1024, 1, 0, 0, 0, 4}, {0, 2, 1, 1024, 1, 0, 0, 0, 8}, {0, 2, 1, 8192, 1, 0, 0, 0, 8},
        {0, 2, 1, 1024, 1, 0, 0, 0, 16}, {0, 2, 4, 1024, 1, 0, 0, 0, 8},
    };
    // matrix-free Hubbard: xcd (remap), nontemporal, wide, tile (down states
    // per tile of the up pass), shfl (hop loop).  The down pass with each
    // slab's column slice staged in LDS (lds = 1) is left out: on the ring
    // L=14 at nb=32 it takes twice the time of the direct gathers, whose
    // slab slice already stays in L2; it remains selectable by fd_spmmv_tune.
    const SpmmvTune mf_cands[] = {
        {0, 0, 1, 0, 1, 0, 16, 1}, {0, 0, 1, 0, 1, 0, 64, 1},  {0, 0, 1, 0, 1, 0, 256, 1},
        {0, 1, 1, 0, 1, 0, 4, 1},  {0, 1, 1, 0, 1, 0, 16, 1},  {0, 1, 1, 0, 1, 0, 64, 1},
        {0, 1, 1, 0, 0, 0, 16, 1}, {0, 0, 1, 0, 0, 0, 64, 1},  {0, 1, 1, 0, 1, 1, 16, 1},
        {0, 0, 1, 0, 1, 0, 64, 2}, {0, 1, 1, 0, 1, 0, 16, 2},  {0, 0, 1, 0, 1, 0, 64, 0},
        {0, 1, 1, 0, 1, 0, 16, 0},
    };
    const SpmmvTune *cb = M.matfree ? mf_cands : cands;
    const SpmmvTune *ce = M.matfree ? mf_cands + sizeof(mf_cands) / sizeof(mf_cands[0])
                                    : cands + sizeof(cands) / sizeof(cands[0]);
    const int lg = __builtin_ctz((unsigned)nb);
    const int di = dt == FD_F64 ? 0 : 1;
    // timed on the filter's own pair of launches: the recurrence with the
    // two-term V update (MODE 5) and the recurrence alone (MODE 4); two
    // passes over the candidates, each keeping its better time
    SpmmvCall c;
    c.nb = nb;
    c.x = buf; c.ldx = nb;
    c.z = (char *)buf + bytes; c.ldz = nb;
    c.y = (char *)buf + bytes; c.ldy = nb;
    c.v = (char *)buf + 2 * bytes; c.ldv = nb;
    c.a = 0.5; c.b = 0.0; c.ct = 0.5; c.cx = 0.25;
    SpmmvCall c5 = c, c4 = c;
    c5.mode = 5;
    c4.mode = 4;
    // fewer repetitions for large matrices; at least 2 pairs
    const int reps = (int)std::max<int64_t>(2, std::min<int64_t>(10, (int64_t)2e9 / (int64_t)(bytes + 1)));
    const int ncand = (int)(ce - cb);
    std::vector<float> tbest(ncand, 1e30f);
    fd_status st = FD_OK;
    for (int pass = 0; pass < 2 && st == FD_OK; pass++) {
        for (int i = 0; i < ncand; i++) {
            const SpmmvTune &t = cb[i];
            if (t.wide && nb < 16) continue;
            if (t.lpr && (nb != 1 || M.cshift != 0 || M.perm)) continue;
            M.tune[di][lg] = t;
            M.tuned[di][lg] = true;
            st = launch_spmmv(M, dt, c5, s);  // warm-up
            if (st != FD_OK) break;
            if (hipEventRecord(e0, s) != hipSuccess) { st = hip_fail(hipErrorUnknown, "autotune event"); break; }
            for (int r = 0; r < reps && st == FD_OK; r++) {
                st = launch_spmmv(M, dt, c5, s);
                if (st == FD_OK) st = launch_spmmv(M, dt, c4, s);
            }
            if (st != FD_OK) break;
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tbest[i] = std::min(tbest[i], ms);
        }
    }
    SpmmvTune best = spmmv_tune();
    float best_ms = 1e30f;
    for (int i = 0; i < ncand; i++)
        if (tbest[i] < best_ms) {
            best_ms = tbest[i];
            best = cb[i];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    M.tune[di][lg] = best;
    M.tuned[di][lg] = st == FD_OK;
    if (best_out) *best_out = best;
    return st;
}

fd_status launch_spmmv(const DevMatrix &M, fd_dtype dt, const SpmmvCall &c, hipStream_t s) {
    // wide: 32 bytes per lane (two 16-byte loads per gathered row segment)
    const int lg = __builtin_ctz((unsigned)std::max(1, c.nb));
    const int di = dt == FD_F64 ? 0 : 1;
    const SpmmvTune &tn = M.tuned[di][lg & 7] ? M.tune[di][lg & 7] : spmmv_tune();
    if (M.matfree) return launch_spmmv_mf(M, dt, c, tn, s);
    if (tn.wide) {
        if (dt == FD_F64) {
            if (c.nb == 64) return launch_t<double, 4, 16>(M, M.val64, c, s);
            if (c.nb == 32) return launch_t<double, 4, 8>(M, M.val64, c, s);
            if (c.nb == 16) return launch_t<double, 4, 4>(M, M.val64, c, s);
        } else {
            if (c.nb == 64) return launch_t<float, 8, 8>(M, M.val32, c, s);
            if (c.nb == 32) return launch_t<float, 8, 4>(M, M.val32, c, s);
            if (c.nb == 16) return launch_t<float, 8, 2>(M, M.val32, c, s);
        }
    }
    if (c.nb == 1 && tn.lpr > 0 && M.cshift == 0 && !M.perm) {
        // one vector: lpr lanes per row (vector-CSR loop)
        if (dt == FD_F64) {
            if (tn.lpr == 4) return launch_t<double, 1, 4, true>(M, M.val64, c, s);
            if (tn.lpr == 8) return launch_t<double, 1, 8, true>(M, M.val64, c, s);
            if (tn.lpr == 16) return launch_t<double, 1, 16, true>(M, M.val64, c, s);
        } else {
            if (tn.lpr == 4) return launch_t<float, 1, 4, true>(M, M.val32, c, s);
            if (tn.lpr == 8) return launch_t<float, 1, 8, true>(M, M.val32, c, s);
            if (tn.lpr == 16) return launch_t<float, 1, 16, true>(M, M.val32, c, s);
        }
    }
    if (dt == FD_F64) {
        switch (c.nb) {
            case 1: return launch_t<double, 1, 1>(M, M.val64, c, s);
            case 2: return launch_t<double, 2, 1>(M, M.val64, c, s);
            case 4: return launch_t<double, 2, 2>(M, M.val64, c, s);
            case 8: return launch_t<double, 2, 4>(M, M.val64, c, s);
            case 16: return launch_t<double, 2, 8>(M, M.val64, c, s);
            case 32: return launch_t<double, 2, 16>(M, M.val64, c, s);
            case 64: return launch_t<double, 2, 32>(M, M.val64, c, s);
        }
    } else {
        switch (c.nb) {
            case 1: return launch_t<float, 1, 1>(M, M.val32, c, s);
            case 2: return launch_t<float, 2, 1>(M, M.val32, c, s);
            case 4: return launch_t<float, 4, 1>(M, M.val32, c, s);
            case 8: return launch_t<float, 4, 2>(M, M.val32, c, s);
            case 16: return launch_t<float, 4, 4>(M, M.val32, c, s);
            case 32: return launch_t<float, 4, 8>(M, M.val32, c, s);
            case 64: return launch_t<float, 4, 16>(M, M.val32, c, s);
        }
    }
    return fail(FD_ERR_INVALID, "nb must be one of 1, 2, 4, 8, 16, 32, 64");
}

}  // namespace fd
