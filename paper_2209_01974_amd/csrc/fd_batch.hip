// Batched sparse kernels on gfx950: many independent FD problems stacked as
// one block-diagonal CSR matrix.  Instance i owns rows [off_i, off_{i+1}),
// its columns are shifted by off_i, and it brings its own scaling
// (alpha_i, beta_i, Alg. 2 caption), filter coefficients mu_i and degree n_i.
// One launch per degree step serves every instance and every bundle, so
// small problems share the GPU instead of each paying for its own launches.
// Rows of an instance whose degree is below the step return at once.
//
// Lane mapping as in the single-matrix kernel: a row of nb values is split
// over G lanes of VEC values (16 bytes); blockIdx.y selects the bundle.
// With 4 or more lanes per row, the row's first 4 or 8 lanes load that many
// entries at once and pass them on by cross-lane permute.
// Row groups are dealt to the 8 XCDs in interleaved chunks of rows (a power
// of two, 1024 by default, chosen per dtype and nb by fd_batch_autotune), so
// that the near neighbours of a row (+-1, +-L for a 3D stencil) stay in one
// XCD's L2.
#include <type_traits>

#include "fd_internal.h"

namespace fd {
namespace {

template <typename T, int VEC> struct BV;
template <> struct BV<double, 1> { typedef double type; };
template <> struct BV<double, 2> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct BV<float, 1> { typedef float type; };
template <> struct BV<float, 2> { typedef float __attribute__((ext_vector_type(2))) type; };
template <> struct BV<float, 4> { typedef float __attribute__((ext_vector_type(4))) type; };

template <typename T>
struct BArgs {
    int64_t D;
    int32_t k, mstride;
    int32_t maxlen;  // longest row of the union
    int32_t uniform;  // every row holds maxlen entries
    int32_t cb_shift;  // log2(blocks per XCD chunk)
    const uint32_t *__restrict__ ptr;
    const uint32_t *__restrict__ col;
    const T *__restrict__ val;
    const uint16_t *__restrict__ inst;
    const double *__restrict__ alpha;
    const double *__restrict__ beta;
    const int32_t *__restrict__ deg;
    const int32_t *__restrict__ act;
    const double *__restrict__ mu;
    const T *x; int64_t ldx, bx;
    T *y; int64_t ldy, by;
    const T *z; int64_t ldz, bz;
    T *v; int64_t ldv, bv;
};

template <typename V>
__device__ __forceinline__ V ldg(const void *p) { return *reinterpret_cast<const V *>(p); }
template <typename V>
__device__ __forceinline__ V ldn(const void *p) { return __builtin_nontemporal_load(reinterpret_cast<const V *>(p)); }
template <typename V>
__device__ __forceinline__ void stn(void *p, V x) { __builtin_nontemporal_store(x, reinterpret_cast<V *>(p)); }
// acc + a x, one rounding per element in every form of the entry loop
template <typename V, typename T>
__device__ __forceinline__ V fmab(T a, V x, V acc) { return __builtin_elementwise_fma((V)a, x, acc); }

// MODE 0: y = A x (rows of active instances)
// MODE 1: y = alpha_i A x + beta_i x
// MODE 2: t = 2 alpha_i A x + 2 beta_i x - v; y = t; v = mu_i0 v + mu_i1 x + mu_i2 t
// MODE 3: t = 2 alpha_i A x + 2 beta_i x - z; y = t (in place over z); v += mu_ik t
// MODE 5: as MODE 3, but V is updated every other step with two terms: at
//   even k, v += mu_i,k-1 x + mu_ik t (x = the previous step's vector); at
//   odd k only when k is the instance's last step (v += mu_ik t)
// SH: entry loop with 4 or more lanes per row; 1 permute rounds of 4
// entries, 2 rounds of 8 (8 or more lanes per row).
// UNI: every row of the union holds p.maxlen entries (no wave exchange)
template <typename T, int VEC, int G, int MODE, int SH, bool UNI>
__global__ __launch_bounds__(256) void k_batch(BArgs<T> p) {
    typedef typename BV<T, VEC>::type V;
    constexpr int RPB = 256 / G;
    // block -> row group: XCD x = b % 8 works through chunks x, x+8, ...
    // (a chunk is 2^cb_shift blocks)
    const int64_t b = blockIdx.x;
    const int64_t j = b >> 3, c = j >> p.cb_shift;
    const int64_t rg = ((((c << 3) + (b & 7))) << p.cb_shift) + (j - (c << p.cb_shift));
    const int64_t row = rg * RPB + threadIdx.x / G;
    bool live = row < p.D;
    const int i = live ? p.inst[row] : 0;
    if constexpr (MODE == 0) {
        live = live && p.act[i];
    } else {
        live = live && p.k <= p.deg[i];
    }
    uint32_t j0, j1;
    int32_t wl;
    if constexpr (G < 4 || UNI) {
        // no exchange between the rows of the wave (no permute rounds, or
        // rows of one length: the rounds run to maxlen)
        if (!live) return;
        j0 = p.ptr[row];
        j1 = p.ptr[row + 1];
        wl = G >= 4 ? p.maxlen : (int32_t)(j1 - j0);
    } else {
        j0 = live ? p.ptr[row] : 0;
        j1 = live ? p.ptr[row + 1] : 0;
        // rounds of the permute loop: the longest live row of this wave (every
        // lane of the wave is still here; lanes of a row share its length)
        wl = (int32_t)(j1 - j0);
#pragma unroll
        for (int o = G; o < 64; o <<= 1) wl = max(wl, __shfl_xor(wl, o, 64));
        // the same value in every lane: a scalar, so the round loop is scalar
        wl = __builtin_amdgcn_readfirstlane(min(wl, p.maxlen));
        if (!live) return;
    }
    const int q = threadIdx.x % G;
    const int64_t bnd = blockIdx.y;
    const T *xq = p.x + bnd * p.bx + q * VEC;
    V zi = (V)0, vi = (V)0;
    T *vr = nullptr;
    bool upd = MODE == 2 || MODE == 3;
    if constexpr (MODE == 5) upd = !(p.k & 1) || p.k == p.deg[i];
    if (upd) {
        vr = p.v + bnd * p.bv + row * p.ldv + q * VEC;
        vi = ldn<V>(vr);
    }
    if constexpr (MODE >= 3) zi = ldn<V>(p.z + bnd * p.bz + row * p.ldz + q * VEC);
    V xi = (V)0;
    if constexpr (MODE != 0) xi = ldg<V>(xq + row * p.ldx);
    V acc0 = (V)0, acc1 = (V)0;
    if constexpr (G >= 4) {
        // rounds of LW entries: lanes 0..LW-1 of the row load one each, the
        // row's lanes take them by permute; the rounds run to the longest
        // row of the wave, so all lanes of a live row take part in every
        // permute (a row's lanes return together, and a permute reads only
        // lanes of its own row)
        constexpr int LW = (G >= 8 && SH == 2) ? 8 : 4;
        const uint32_t len = j1 - j0;
        const int rbase = (int)(threadIdx.x & 63) - q;
        for (int r0 = 0; r0 < wl; r0 += LW) {
            const uint32_t jq = (uint32_t)(r0 + q);
            uint32_t cm = 0;
            T am = (T)0;
            if (q < LW && jq < len) {
                cm = p.col[j0 + jq];
                am = p.val[j0 + jq];
            }
            uint32_t cc[LW];
            T aa[LW];
#pragma unroll
            for (int u = 0; u < LW; u++) {
                cc[u] = (uint32_t)__shfl((int)cm, rbase + u, 64);
                aa[u] = __shfl(am, rbase + u, 64);
            }
            V xs[LW];
#pragma unroll
            for (int u = 0; u < LW; u++) xs[u] = ((uint32_t)(r0 + u) < len) ? ldg<V>(xq + (int64_t)cc[u] * p.ldx) : (V)0;
#pragma unroll
            for (int u = 0; u < LW; u++)
                if ((uint32_t)(r0 + u) < len) {
                    if (u & 1) acc1 = fmab(aa[u], xs[u], acc1);
                    else acc0 = fmab(aa[u], xs[u], acc0);
                }
        }
    } else {
        uint32_t jj = j0;
        for (; jj + 2 <= j1; jj += 2) {
            const uint32_t c0 = p.col[jj], c1 = p.col[jj + 1];
            const T e0 = p.val[jj], e1 = p.val[jj + 1];
            acc0 = fmab(e0, ldg<V>(xq + (int64_t)c0 * p.ldx), acc0);
            acc1 = fmab(e1, ldg<V>(xq + (int64_t)c1 * p.ldx), acc1);
        }
        if (jj < j1) acc0 = fmab(p.val[jj], ldg<V>(xq + (int64_t)p.col[jj] * p.ldx), acc0);
    }
    const V acc = acc0 + acc1;
    T *yr = p.y + bnd * p.by + row * p.ldy + q * VEC;
    if constexpr (MODE == 0) {
        stn<V>(yr, acc);
    } else {
        const double sc = MODE == 1 ? 1.0 : 2.0;
        const T a = (T)(sc * p.alpha[i]), bb = (T)(sc * p.beta[i]);
        V t = a * acc + bb * xi;
        if constexpr (MODE == 1) {
            stn<V>(yr, t);
        } else if constexpr (MODE == 2) {
            const double *m = p.mu + (int64_t)i * p.mstride;
            t -= vi;
            stn<V>(yr, t);
            stn<V>(vr, (T)m[0] * vi + (T)m[1] * xi + (T)m[2] * t);
        } else if constexpr (MODE == 3) {
            t -= zi;
            stn<V>(yr, t);
            stn<V>(vr, vi + (T)p.mu[(int64_t)i * p.mstride + p.k] * t);
        } else {
            const double *m = p.mu + (int64_t)i * p.mstride;
            t -= zi;
            stn<V>(yr, t);
            if (p.k & 1) {
                if (upd) stn<V>(vr, vi + (T)m[p.k] * t);
            } else {
                stn<V>(vr, vi + (T)m[p.k - 1] * xi + (T)m[p.k] * t);
            }
        }
    }
}

template <typename T, int VEC, int G, int SH, bool UNI>
fd_status launch_bu(const BArgs<T> &p, const BatchCall &c, const dim3 &grid, hipStream_t s) {
    switch (c.mode) {
        case 0: hipLaunchKernelGGL((k_batch<T, VEC, G, 0, SH, UNI>), grid, dim3(256), 0, s, p); break;
        case 1: hipLaunchKernelGGL((k_batch<T, VEC, G, 1, SH, UNI>), grid, dim3(256), 0, s, p); break;
        case 2: hipLaunchKernelGGL((k_batch<T, VEC, G, 2, SH, UNI>), grid, dim3(256), 0, s, p); break;
        case 3: hipLaunchKernelGGL((k_batch<T, VEC, G, 3, SH, UNI>), grid, dim3(256), 0, s, p); break;
        case 5: hipLaunchKernelGGL((k_batch<T, VEC, G, 5, SH, UNI>), grid, dim3(256), 0, s, p); break;
        default: return fail(FD_ERR_INVALID, "batched SpMMV: bad mode");
    }
    FD_HIP(hipGetLastError());
    return FD_OK;
}

template <typename T, int VEC, int G, int SH>
fd_status launch_bs(const BatchDev &B, const BArgs<T> &p, const BatchCall &c, const dim3 &grid, hipStream_t s) {
    (void)B;
    if (G >= 4 && p.uniform) return launch_bu<T, VEC, G, SH, true>(p, c, grid, s);
    return launch_bu<T, VEC, G, SH, false>(p, c, grid, s);
}

template <typename T, int VEC, int G>
fd_status launch_bt(const BatchDev &B, const T *val, const BatchCall &c, hipStream_t s) {
    constexpr int RPB = 256 / G;
    BArgs<T> p;
    p.D = B.D;
    p.k = c.k;
    p.mstride = B.mstride;
    p.maxlen = B.maxlen;
    p.uniform = B.minlen == B.maxlen ? 1 : 0;
    p.ptr = B.ptr; p.col = B.col; p.val = val; p.inst = B.inst;
    p.alpha = B.alpha; p.beta = B.beta; p.deg = B.deg; p.act = B.act; p.mu = B.mu;
    p.x = (const T *)c.x; p.ldx = c.ldx; p.bx = c.bx;
    p.y = (T *)c.y; p.ldy = c.ldy; p.by = c.by;
    p.z = (const T *)c.z; p.ldz = c.ldz; p.bz = c.bz;
    p.v = (T *)c.v; p.ldv = c.ldv; p.bv = c.bv;
    if (B.D == 0) return FD_OK;
    // launch shape of this dtype and nb: XCD chunk (rows) and entry loop
    const int di = std::is_same<T, double>::value ? 0 : 1, lg = __builtin_ctz((unsigned)c.nb);
    const int64_t chunk = B.chunk[di][lg] > 0 ? B.chunk[di][lg] : 1024;
    const int64_t cb = std::max<int64_t>(1, chunk / RPB);  // blocks per chunk (a power of two)
    p.cb_shift = __builtin_ctzll((unsigned long long)cb);
    // grid: whole super-chunks (8 chunks of cb blocks), so the block -> row
    // group map is a bijection; row groups past D return at once
    const int64_t ngroups = (B.D + RPB - 1) / RPB;
    const int64_t super = 8 * cb;
    const int64_t nblk = (ngroups + super - 1) / super * super;
    if (nblk > 0x7fffffff || c.nbundles < 1 || c.nbundles > 65535)
        return fail(FD_ERR_UNSUPPORTED, "batched SpMMV: grid too large");
    const dim3 grid((unsigned)nblk, c.nbundles);
    if constexpr (G >= 8) {
        if (B.sh[di][lg] == 1) return launch_bs<T, VEC, G, 1>(B, p, c, grid, s);
    }
    return launch_bs<T, VEC, G, 2>(B, p, c, grid, s);
}

}  // namespace

fd_status launch_batch(const BatchDev &B, fd_dtype dt, const BatchCall &c, hipStream_t s) {
    if (dt == FD_F64) {
        switch (c.nb) {
            case 1: return launch_bt<double, 1, 1>(B, B.val64, c, s);
            case 2: return launch_bt<double, 2, 1>(B, B.val64, c, s);
            case 4: return launch_bt<double, 2, 2>(B, B.val64, c, s);
            case 8: return launch_bt<double, 2, 4>(B, B.val64, c, s);
            case 16: return launch_bt<double, 2, 8>(B, B.val64, c, s);
            case 32: return launch_bt<double, 2, 16>(B, B.val64, c, s);
            case 64: return launch_bt<double, 2, 32>(B, B.val64, c, s);
        }
    } else {
        switch (c.nb) {
            case 1: return launch_bt<float, 1, 1>(B, B.val32, c, s);
            case 2: return launch_bt<float, 2, 1>(B, B.val32, c, s);
            case 4: return launch_bt<float, 4, 1>(B, B.val32, c, s);
            case 8: return launch_bt<float, 4, 2>(B, B.val32, c, s);
            case 16: return launch_bt<float, 4, 4>(B, B.val32, c, s);
            case 32: return launch_bt<float, 4, 8>(B, B.val32, c, s);
            case 64: return launch_bt<float, 4, 16>(B, B.val32, c, s);
        }
    }
    return fail(FD_ERR_INVALID, "nb must be one of 1, 2, 4, 8, 16, 32, 64");
}

}  // namespace fd
