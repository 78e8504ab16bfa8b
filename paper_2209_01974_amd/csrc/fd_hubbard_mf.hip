// Matrix-free Hubbard SpMMV and fused Chebyshev step on gfx950.
//
// In the up-major Fock basis (row (a, b) = a nd + b) the Hubbard ring is the
// tensor-product sum H = H_up x I + I x H_dn + U D (the structure the paper's
// matrix-free Hubbard SpMV uses, Sec. 4.2): row (a, b) couples to (a', b) for
// each up hop a -> a' and to (a, b') for each down hop b -> b'.  No matrix is
// stored.  The operator is applied in two passes so that both kinds of
// gathers are served from cache:
//   pass 1, rows in natural order: the down hops and the diagonal.  The
//     gathers of row (a, b) stay in the slab x[a, :] (nd rows), which L2
//     holds.  It writes the part of the update that needs no up hop,
//     e.g. y = a (I x H_dn + U D) x + b x - z for the Chebyshev step.
//   pass 2, rows in tiles of tile_b down-states, tile after tile with all up
//     states of a tile in a row: y += a (H_up x I) x, then the rest of the
//     update.  The gathers x[a', b] of one tile touch only nu * tile_b rows.
// The first pass writes its partial result into y itself, so the only extra
// traffic over a stored-matrix step is one more read and write of y, against
// the matrix and the strided up-hop gathers it saves.  Lane mapping as in
// the stored-matrix kernel: a row of nb values is split over G lanes of VEC
// values each; blockIdx.y selects the bundle.  With 4 or more lanes per row
// the row's first 4 or 8 lanes load that many hops (target, element) at once
// and pass them on by cross-lane permute.
#include "fd_internal.h"

namespace fd {
namespace {

template <typename T, int VEC> struct VT;
template <> struct VT<double, 1> { typedef double type; };
template <> struct VT<double, 2> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct VT<float, 1> { typedef float type; };
template <> struct VT<float, 2> { typedef float __attribute__((ext_vector_type(2))) type; };
template <> struct VT<float, 4> { typedef float __attribute__((ext_vector_type(4))) type; };
template <> struct VT<double, 4> { typedef double __attribute__((ext_vector_type(4))) type; };
template <> struct VT<float, 8> { typedef float __attribute__((ext_vector_type(8))) type; };

template <typename T>
struct MfArgs {
    int64_t nu, nd, D, nlog;  // nlog: logical rows of pass 2 (ntiles nu tile_b)
    int64_t tile_b;
    int64_t nblk, q8;         // blocks per bundle, floor(nblk / 8)
    int32_t maxu, maxd;       // most hops of an up / down state
    const uint64_t *__restrict__ mu;
    const uint64_t *__restrict__ md;
    const int32_t *__restrict__ off_u;
    const int32_t *__restrict__ idx_u;
    const T *__restrict__ val_u;
    const int32_t *__restrict__ off_d;
    const int32_t *__restrict__ idx_d;
    const T *__restrict__ val_d;
    const uint16_t *__restrict__ hop16_d;  // down hops packed: target | 0x8000 for +tmag
    T tmag;                                // |element| of every down hop
    T U;
    const T *x; int64_t ldx, bx;
    T *y; int64_t ldy, by;
    const T *z; int64_t ldz, bz;
    T *v; int64_t ldv, bv;
    T a, b, cv, cx, ct;
};

template <typename V>
__device__ __forceinline__ V ld(const void *p) { return *reinterpret_cast<const V *>(p); }
// acc + e x with one rounding per element in every form of the hop loop
template <typename V, typename T>
__device__ __forceinline__ V fmah(T e, V x, V acc) { return __builtin_elementwise_fma((V)e, x, acc); }

// Hops h of one row, h = 0 .. len-1 at tables idx[j0 + h], val[j0 + h]: the
// gathered row of hop h is xq + (base + idx * stride) * ldx.  Even hops go
// to acc0, odd ones to acc1.  SH 1 / 2: lanes 0..LW-1 of the row (LW = 4 /
// 8, q < LW) load one hop each per round and the row's lanes take them by
// permute; the rounds run to maxlen, the most hops of any row in the wave
// (wave_len), so that every lane of a live row takes part in every permute.  SH 0: every lane
// loads every hop (broadcast).
template <typename T, typename V, int G, int SH>
__device__ __forceinline__ void hop_sum(const int32_t *__restrict__ idx, const T *__restrict__ val, int32_t j0,
                                        int32_t len, int32_t maxlen, const T *xq, int64_t base, int64_t stride,
                                        int64_t ldx, int q, V &acc0, V &acc1) {
    if constexpr (SH != 0) {
        constexpr int LW = SH == 2 ? 8 : 4;
        static_assert(G >= LW, "a load round needs LW lanes per row");
        const int rbase = (int)(threadIdx.x & 63) - q;
        for (int r0 = 0; r0 < maxlen; r0 += LW) {
            int32_t cm = 0;
            T em = (T)0;
            if (q < LW && r0 + q < len) {
                cm = idx[j0 + r0 + q];
                em = val[j0 + r0 + q];
            }
            int32_t cc[LW];
            T ee[LW];
#pragma unroll
            for (int u = 0; u < LW; u++) {
                cc[u] = __shfl(cm, rbase + u, 64);
                ee[u] = __shfl(em, rbase + u, 64);
            }
            V xs[LW];
#pragma unroll
            for (int u = 0; u < LW; u++) xs[u] = (r0 + u < len) ? ld<V>(xq + (base + (int64_t)cc[u] * stride) * ldx) : (V)0;
#pragma unroll
            for (int u = 0; u < LW; u++)
                if (r0 + u < len) {
                    if (u & 1) acc1 = fmah(ee[u], xs[u], acc1);
                    else acc0 = fmah(ee[u], xs[u], acc0);
                }
        }
    } else {
        int32_t h = 0;
        // four hops per round, all loads of a round independent
        for (; h + 4 <= len; h += 4) {
            const int32_t c0 = idx[j0 + h], c1 = idx[j0 + h + 1], c2 = idx[j0 + h + 2], c3 = idx[j0 + h + 3];
            const T e0 = val[j0 + h], e1 = val[j0 + h + 1], e2 = val[j0 + h + 2], e3 = val[j0 + h + 3];
            const V x0 = ld<V>(xq + (base + (int64_t)c0 * stride) * ldx);
            const V x1 = ld<V>(xq + (base + (int64_t)c1 * stride) * ldx);
            const V x2 = ld<V>(xq + (base + (int64_t)c2 * stride) * ldx);
            const V x3 = ld<V>(xq + (base + (int64_t)c3 * stride) * ldx);
            acc0 = fmah(e0, x0, acc0);
            acc1 = fmah(e1, x1, acc1);
            acc0 = fmah(e2, x2, acc0);
            acc1 = fmah(e3, x3, acc1);
        }
        // at most three hops left (h is a multiple of 4): even, odd, even
        if (h < len) acc0 = fmah(val[j0 + h], ld<V>(xq + (base + (int64_t)idx[j0 + h] * stride) * ldx), acc0);
        if (h + 1 < len)
            acc1 = fmah(val[j0 + h + 1], ld<V>(xq + (base + (int64_t)idx[j0 + h + 1] * stride) * ldx), acc1);
        if (h + 2 < len)
            acc0 = fmah(val[j0 + h + 2], ld<V>(xq + (base + (int64_t)idx[j0 + h + 2] * stride) * ldx), acc0);
    }
}
// Rounds of the permute hop loop: the most hops of any row in this wave
// (lanes of a row share len; every lane of the wave must call this).
template <int G, int SH>
__device__ __forceinline__ int32_t wave_len(int32_t len, int32_t maxlen) {
    if constexpr (SH == 0) {
        return len;
    } else {
        int32_t w = len;
#pragma unroll
        for (int o = G; o < 64; o <<= 1) w = max(w, __shfl_xor(w, o, 64));
        // the same value in every lane: a scalar, so the round loop is scalar
        return __builtin_amdgcn_readfirstlane(min(w, maxlen));
    }
}

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

// Block index -> logical block.  XCD: the hardware deals consecutive blocks
// to the 8 XCDs in turn; remap so that XCD k works through the k-th eighth
// of the logical blocks (a bijection on the first 8 q8 blocks, the tail
// unchanged), which keeps a slab or a tile in one XCD's L2.
template <bool XCD>
__device__ __forceinline__ int64_t logical_block(int64_t bid, int64_t q8) {
    if constexpr (XCD) {
        if (bid < 8 * q8) return (bid & 7) * q8 + (bid >> 3);
    }
    return bid;
}

// pass 1: down hops + diagonal, rows in natural order.
//   MODE 0: y = s           MODE 1: y = a s + b x
//   MODE 2: y = a s + b x - v        MODE 3, 4, 5: y = a s + b x - z
// with s = (I x H_dn + U D) x.  y may alias z (same element read first).
template <typename T, int VEC, int G, int MODE, bool XCD, bool NT, int SH>
__global__ __launch_bounds__(256) void k_mf_down(MfArgs<T> p) {
    typedef typename VT<T, VEC>::type V;
    constexpr int RPB = 256 / G;
    const int64_t blk = logical_block<XCD>(blockIdx.x, p.q8);
    const int64_t s = blk * RPB + threadIdx.x / G;
    const bool live = s < p.D;
    // D < 2^32 (checked at build): 32-bit division, far cheaper than 64-bit
    const int64_t a = live ? (uint32_t)s / (uint32_t)p.nd : 0, b = live ? s - a * p.nd : 0;
    const int32_t j0 = live ? p.off_d[b] : 0;
    const int32_t len = live ? p.off_d[b + 1] - j0 : 0;
    const int32_t wl = wave_len<G, SH>(len, p.maxd);
    if (!live) return;
    const int q = threadIdx.x % G;
    const int64_t bnd = blockIdx.y;
    const T *xq = p.x + bnd * p.bx + q * VEC;
    V zi = (V)0;
    if constexpr (MODE == 2) zi = lds<V, NT>(p.v + bnd * p.bv + s * p.ldv + q * VEC);
    if constexpr (MODE >= 3) zi = lds<V, NT>(p.z + bnd * p.bz + s * p.ldz + q * VEC);
    const V xi = ld<V>(xq + s * p.ldx);
    V acc0 = (p.U * (T)__popcll(p.mu[a] & p.md[b])) * xi, acc1 = (V)0;
    hop_sum<T, V, G, SH>(p.idx_d, p.val_d, j0, len, wl, xq, a * p.nd, 1, p.ldx, q, acc0, acc1);
    V r = acc0 + acc1;
    if constexpr (MODE >= 1) r = p.a * r + p.b * xi;
    if constexpr (MODE >= 2) r -= zi;
    sts<V, NT>(p.y + bnd * p.by + s * p.ldy + q * VEC, r);
}

// pass 2: up hops, rows in down-state tiles; t = y + c u with
// u = (H_up x I) x and c = 1 (MODE 0) or a (else).  Then
//   MODE 0, 1, 4: y = t
//   MODE 2: y = t, v = cv v + cx x + ct t
//   MODE 3: y = t, v = v + ct t
//   MODE 5: y = t, v = v + cx x + ct t
template <typename T, int VEC, int G, int MODE, bool XCD, bool NT, int SH>
__global__ __launch_bounds__(256) void k_mf_up(MfArgs<T> p) {
    typedef typename VT<T, VEC>::type V;
    constexpr int RPB = 256 / G;
    const int64_t blk = logical_block<XCD>(blockIdx.x, p.q8);
    const int64_t l = blk * RPB + threadIdx.x / G;
    const int64_t per_tile = p.nu * p.tile_b;
    int64_t tile = 0, a = 0;
    if (l < p.nlog) {
        if (p.nlog < (int64_t(1) << 32)) {  // uniform branch: 32-bit divisions
            tile = (uint32_t)l / (uint32_t)per_tile;
            a = (uint32_t)(l - tile * per_tile) / (uint32_t)p.tile_b;
        } else {
            tile = l / per_tile;
            a = (l - tile * per_tile) / p.tile_b;
        }
    }
    const int64_t b = tile * p.tile_b + (l - tile * per_tile - a * p.tile_b);
    const bool live = l < p.nlog && b < p.nd;
    const int32_t j0 = live ? p.off_u[a] : 0;
    const int32_t len = live ? p.off_u[a + 1] - j0 : 0;
    const int32_t wl = wave_len<G, SH>(len, p.maxu);
    if (!live) return;
    const int64_t s = a * p.nd + b;
    const int q = threadIdx.x % G;
    const int64_t bnd = blockIdx.y;
    const T *xq = p.x + bnd * p.bx + q * VEC;
    T *yr = p.y + bnd * p.by + s * p.ldy + q * VEC;
    V vi = (V)0, xi = (V)0;
    T *vr = nullptr;
    if constexpr (MODE == 2 || MODE == 3 || MODE == 5) {
        vr = p.v + bnd * p.bv + s * p.ldv + q * VEC;
        vi = lds<V, NT>(vr);
    }
    if constexpr (MODE == 2 || MODE == 5) xi = ld<V>(xq + s * p.ldx);
    const V yi = lds<V, NT>(yr);
    V acc0 = (V)0, acc1 = (V)0;
    hop_sum<T, V, G, SH>(p.idx_u, p.val_u, j0, len, wl, xq, b, p.nd, p.ldx, q, acc0, acc1);
    V t;
    if constexpr (MODE == 0) t = yi + (acc0 + acc1);
    else t = yi + p.a * (acc0 + acc1);
    sts<V, NT>(yr, t);
    if constexpr (MODE == 2) sts<V, NT>(vr, p.cv * vi + p.cx * xi + p.ct * t);
    if constexpr (MODE == 3) sts<V, NT>(vr, vi + p.ct * t);
    if constexpr (MODE == 5) sts<V, NT>(vr, vi + p.cx * xi + p.ct * t);
}

// pass 1 with the slab staged in LDS (the x-gather of the down hops served
// from LDS): one block per (up configuration a, 16-byte column slice of the
// bundle).  The block first issues its rows' streamed loads (z or v), then
// copies the slab's slice x[a, 0..nd-1, slice] into LDS (one 16-byte load
// per row), and after one barrier every row (a, b) of the slab takes the
// diagonal and its down hops from LDS.  The G slices of a slab are dealt to
// one XCD one after another, so each row of the slab comes from HBM once and
// from L2 for the other slices.  Down-hop targets and signs come from a
// packed 16-bit table (all down hops have the same magnitude).  Same
// arithmetic, in the same order, as k_mf_down: bitwise equal results.
constexpr int LDS_THREADS = 512;
constexpr int LDS_RB = 8;  // rows per thread and round (nd <= 4096: one round)
template <typename T, int VEC, int G, int MODE, bool NT>
__global__ __launch_bounds__(LDS_THREADS) void k_mf_down_lds(MfArgs<T> p) {
    typedef typename VT<T, VEC>::type V;
    extern __shared__ unsigned char smem[];
    V *xs = reinterpret_cast<V *>(smem);
    const int64_t blk = blockIdx.x;
    const int64_t j = blk >> 3;
    const int64_t a = (j / G) * 8 + (blk & 7);
    const int sl = (int)(j % G);
    if (a >= p.nu) return;  // the whole block leaves before its barrier
    const int64_t bnd = blockIdx.y;
    const int64_t nd = p.nd, r0 = a * nd;
    const int t = threadIdx.x;
    const T *xq = p.x + bnd * p.bx + sl * VEC;
    const uint64_t ma = p.mu[a];
    for (int64_t base = 0; base < nd; base += (int64_t)LDS_THREADS * LDS_RB) {
        V zr[LDS_RB];
#pragma unroll
        for (int u = 0; u < LDS_RB; u++) {
            const int64_t b = base + (int64_t)u * LDS_THREADS + t;
            zr[u] = (V)0;
            if (b < nd) {
                if constexpr (MODE == 2) zr[u] = lds<V, NT>(p.v + bnd * p.bv + (r0 + b) * p.ldv + sl * VEC);
                if constexpr (MODE >= 3) zr[u] = lds<V, NT>(p.z + bnd * p.bz + (r0 + b) * p.ldz + sl * VEC);
            }
        }
        if (base == 0) {
            for (int64_t b = t; b < nd; b += LDS_THREADS) xs[b] = ld<V>(xq + (r0 + b) * p.ldx);
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < LDS_RB; u++) {
            const int64_t b = base + (int64_t)u * LDS_THREADS + t;
            if (b >= nd) break;
            const V xi = xs[b];
            V acc0 = (p.U * (T)__popcll(ma & p.md[b])) * xi, acc1 = (V)0;
            const int32_t h1 = p.off_d[b + 1];
            int32_t h = p.off_d[b];
            for (; h + 2 <= h1; h += 2) {
                const uint32_t e0 = p.hop16_d[h], e1 = p.hop16_d[h + 1];
                acc0 = fmah((e0 & 0x8000u) ? p.tmag : -p.tmag, xs[e0 & 0x7fffu], acc0);
                acc1 = fmah((e1 & 0x8000u) ? p.tmag : -p.tmag, xs[e1 & 0x7fffu], acc1);
            }
            if (h < h1) {
                const uint32_t e0 = p.hop16_d[h];
                acc0 = fmah((e0 & 0x8000u) ? p.tmag : -p.tmag, xs[e0 & 0x7fffu], acc0);
            }
            V r = acc0 + acc1;
            if constexpr (MODE >= 1) r = p.a * r + p.b * xi;
            if constexpr (MODE >= 2) r -= zr[u];
            sts<V, NT>(p.y + bnd * p.by + (r0 + b) * p.ldy + sl * VEC, r);
        }
    }
}

template <typename T, int VEC, int G, int MODE, bool XCD, bool NT, int SH>
fd_status launch_mode(const MfArgs<T> &p, int nbund, int64_t g1, int64_t g2, hipStream_t s, bool lds) {
    MfArgs<T> p1 = p, p2 = p;
    p1.nblk = g1;
    p1.q8 = g1 / 8;
    p2.nblk = g2;
    p2.q8 = g2 / 8;
    if (lds) {
        typedef typename VT<T, VEC>::type V;
        const size_t sh = (size_t)p.nd * sizeof(V);
        if (sh > 65536)
            FD_HIP(hipFuncSetAttribute((const void *)k_mf_down_lds<T, VEC, G, MODE, NT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
        const int64_t nb1 = (p.nu + 7) / 8 * 8 * G;
        hipLaunchKernelGGL((k_mf_down_lds<T, VEC, G, MODE, NT>), dim3((unsigned)nb1, nbund), dim3(LDS_THREADS), sh, s,
                           p1);
    } else {
        hipLaunchKernelGGL((k_mf_down<T, VEC, G, MODE, XCD, NT, SH>), dim3((unsigned)g1, nbund), dim3(256), 0, s,
                           p1);
    }
    FD_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_mf_up<T, VEC, G, MODE, XCD, NT, SH>), dim3((unsigned)g2, nbund), dim3(256), 0, s, p2);
    FD_HIP(hipGetLastError());
    return FD_OK;
}

template <typename T, int VEC, int G, bool XCD, bool NT, int SH>
fd_status launch_m(const MfArgs<T> &p, int mode, int nbund, int64_t g1, int64_t g2, hipStream_t s, bool lds) {
    switch (mode) {
        case 0: return launch_mode<T, VEC, G, 0, XCD, NT, SH>(p, nbund, g1, g2, s, lds);
        case 1: return launch_mode<T, VEC, G, 1, XCD, NT, SH>(p, nbund, g1, g2, s, lds);
        case 2: return launch_mode<T, VEC, G, 2, XCD, NT, SH>(p, nbund, g1, g2, s, lds);
        case 3: return launch_mode<T, VEC, G, 3, XCD, NT, SH>(p, nbund, g1, g2, s, lds);
        case 4: return launch_mode<T, VEC, G, 4, XCD, NT, SH>(p, nbund, g1, g2, s, lds);
        case 5: return launch_mode<T, VEC, G, 5, XCD, NT, SH>(p, nbund, g1, g2, s, lds);
    }
    return fail(FD_ERR_INVALID, "matrix-free SpMMV: bad mode");
}

// hop loop: permute rounds of 8 need 8 lanes per row, rounds of 4 need 4;
// with fewer lanes the next smaller form runs
template <typename T, int VEC, int G, bool XCD, bool NT>
fd_status launch_x(const MfArgs<T> &p, int mode, int sh, int nbund, int64_t g1, int64_t g2, hipStream_t s,
                   bool lds) {
    if constexpr (G >= 8) {
        if (sh >= 2) return launch_m<T, VEC, G, XCD, NT, 2>(p, mode, nbund, g1, g2, s, lds);
    }
    if constexpr (G >= 4) {
        if (sh >= 1) return launch_m<T, VEC, G, XCD, NT, 1>(p, mode, nbund, g1, g2, s, lds);
    }
    return launch_m<T, VEC, G, XCD, NT, 0>(p, mode, nbund, g1, g2, s, lds);
}

template <typename T, int VEC, int G>
fd_status launch_mf_t(const DevMatrix &M, const T *val_u, const T *val_d, const SpmmvTune &tn,
                      const SpmmvCall &c, hipStream_t s) {
    constexpr int RPB = 256 / G;
    MfArgs<T> p;
    p.nu = M.nu;
    p.nd = M.nd;
    p.D = M.D;
    p.tile_b = std::max<int64_t>(1, std::min<int64_t>(tn.tile > 0 ? tn.tile : M.mf_tile, M.nd));
    const int64_t ntiles = (M.nd + p.tile_b - 1) / p.tile_b;
    p.nlog = ntiles * M.nu * p.tile_b;
    p.nblk = p.q8 = 0;
    p.maxu = M.mf_maxu;
    p.maxd = M.mf_maxd;
    p.mu = M.mu;
    p.md = M.md;
    p.off_u = M.off_u;
    p.idx_u = M.idx_u;
    p.val_u = val_u;
    p.off_d = M.off_d;
    p.idx_d = M.idx_d;
    p.val_d = val_d;
    p.hop16_d = M.hop16_d;
    p.tmag = (T)M.tmag_d;
    p.U = (T)M.U;
    p.x = (const T *)c.x; p.ldx = c.ldx; p.bx = c.bx;
    p.y = (T *)c.y; p.ldy = c.ldy; p.by = c.by;
    p.z = (const T *)c.z; p.ldz = c.ldz; p.bz = c.bz;
    p.v = (T *)c.v; p.ldv = c.ldv; p.bv = c.bv;
    p.a = (T)c.a; p.b = (T)c.b; p.cv = (T)c.cv; p.cx = (T)c.cx; p.ct = (T)c.ct;
    if (M.D == 0) return FD_OK;
    const int64_t g1 = (M.D + RPB - 1) / RPB, g2 = (p.nlog + RPB - 1) / RPB;
    if (g1 > 0x7fffffff || g2 > 0x7fffffff || c.nbundles < 1 || c.nbundles > 65535)
        return fail(FD_ERR_UNSUPPORTED, "matrix-free SpMMV: grid too large");
    const bool xcd = tn.xcd == 1, nt = tn.nontemporal != 0;
    const int sh = tn.shfl;
    // the LDS-staged down pass: packed down hops and a slab slice that fits
    // in LDS (nd 16-byte rows, at most 160 KB)
    const bool lds = tn.lds != 0 && M.hop16_d != nullptr && M.nd * (int64_t)(VEC * sizeof(T)) <= 160 * 1024;
    if (xcd) {
        if (nt) return launch_x<T, VEC, G, true, true>(p, c.mode, sh, c.nbundles, g1, g2, s, lds);
        return launch_x<T, VEC, G, true, false>(p, c.mode, sh, c.nbundles, g1, g2, s, lds);
    }
    if (nt) return launch_x<T, VEC, G, false, true>(p, c.mode, sh, c.nbundles, g1, g2, s, lds);
    return launch_x<T, VEC, G, false, false>(p, c.mode, sh, c.nbundles, g1, g2, s, lds);
}

}  // namespace

fd_status launch_spmmv_mf(const DevMatrix &M, fd_dtype dt, const SpmmvCall &c, const SpmmvTune &tn,
                          hipStream_t s) {
    if (tn.wide) {  // 32 bytes per lane
        if (dt == FD_F64) {
            if (c.nb == 64) return launch_mf_t<double, 4, 16>(M, M.val_u64, M.val_d64, tn, c, s);
            if (c.nb == 32) return launch_mf_t<double, 4, 8>(M, M.val_u64, M.val_d64, tn, c, s);
            if (c.nb == 16) return launch_mf_t<double, 4, 4>(M, M.val_u64, M.val_d64, tn, c, s);
        } else {
            if (c.nb == 64) return launch_mf_t<float, 8, 8>(M, M.val_u32, M.val_d32, tn, c, s);
            if (c.nb == 32) return launch_mf_t<float, 8, 4>(M, M.val_u32, M.val_d32, tn, c, s);
            if (c.nb == 16) return launch_mf_t<float, 8, 2>(M, M.val_u32, M.val_d32, tn, c, s);
        }
    }
    if (dt == FD_F64) {
        switch (c.nb) {
            case 1: return launch_mf_t<double, 1, 1>(M, M.val_u64, M.val_d64, tn, c, s);
            case 2: return launch_mf_t<double, 2, 1>(M, M.val_u64, M.val_d64, tn, c, s);
            case 4: return launch_mf_t<double, 2, 2>(M, M.val_u64, M.val_d64, tn, c, s);
            case 8: return launch_mf_t<double, 2, 4>(M, M.val_u64, M.val_d64, tn, c, s);
            case 16: return launch_mf_t<double, 2, 8>(M, M.val_u64, M.val_d64, tn, c, s);
            case 32: return launch_mf_t<double, 2, 16>(M, M.val_u64, M.val_d64, tn, c, s);
            case 64: return launch_mf_t<double, 2, 32>(M, M.val_u64, M.val_d64, tn, c, s);
        }
    } else {
        switch (c.nb) {
            case 1: return launch_mf_t<float, 1, 1>(M, M.val_u32, M.val_d32, tn, c, s);
            case 2: return launch_mf_t<float, 2, 1>(M, M.val_u32, M.val_d32, tn, c, s);
            case 4: return launch_mf_t<float, 4, 1>(M, M.val_u32, M.val_d32, tn, c, s);
            case 8: return launch_mf_t<float, 4, 2>(M, M.val_u32, M.val_d32, tn, c, s);
            case 16: return launch_mf_t<float, 4, 4>(M, M.val_u32, M.val_d32, tn, c, s);
            case 32: return launch_mf_t<float, 4, 8>(M, M.val_u32, M.val_d32, tn, c, s);
            case 64: return launch_mf_t<float, 4, 16>(M, M.val_u32, M.val_d32, tn, c, s);
        }
    }
    return fail(FD_ERR_INVALID, "nb must be one of 1, 2, 4, 8, 16, 32, 64");
}

}  // namespace fd
