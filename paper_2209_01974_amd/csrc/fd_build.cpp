// Host-side matrix builders for libfd: generated Hamiltonians -> canonical
// CSR (ascending columns, diagonal always stored) -> optional SELL-C-sigma,
// plus the Gershgorin inclusion interval and the Chebyshev coefficients.
//
// The FD method needs an inclusion interval [lam_l, lam_r] of the spectrum
// for the Chebyshev scaling (Sec. 2) and A stored row-wise with uint32 column
// indices (Sec. 3.1, Eq. traffic with S_i = 4).  Row generation runs on all
// host cores.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "fd_internal.h"

namespace fd {

namespace {

int n_threads() {
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 4;
    return (int)std::min<unsigned>(h, 32);
}

template <class F>
void parallel_for(int64_t n, F &&f) {
    int T = n_threads();
    if (n < 4096) T = 1;
    std::vector<std::thread> th;
    int64_t per = (n + T - 1) / T;
    for (int k = 0; k < T; k++) {
        int64_t lo = k * per, hi = std::min<int64_t>(n, lo + per);
        if (lo >= hi) break;
        th.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    for (auto &x : th) x.join();
}

// binomial table C[n][k], n <= 64
struct Binom {
    uint64_t c[65][65];
    Binom() {
        std::memset(c, 0, sizeof(c));
        for (int n = 0; n <= 64; n++) {
            c[n][0] = 1;
            for (int k = 1; k <= n; k++) c[n][k] = c[n - 1][k - 1] + (k <= n - 1 ? c[n - 1][k] : 0);
        }
    }
};
const Binom &binom() {
    static Binom b;
    return b;
}

// Combinatorial number system: the colex rank of a subset equals the rank of
// its bitmask in increasing integer order.
uint64_t subset_rank(uint64_t m) {
    uint64_t r = 0;
    int i = 1;
    while (m) {
        int p = __builtin_ctzll(m);
        r += binom().c[p][i];
        i++;
        m &= m - 1;
    }
    return r;
}

// next larger integer with the same popcount (Gosper)
uint64_t next_same_popcount(uint64_t v) {
    uint64_t t = v | (v - 1);
    return (t + 1) | (((~t & -~t) - 1) >> (__builtin_ctzll(v) + 1));
}

struct Hop {
    uint32_t rank;
    double el;
};

// For each spin configuration, the configurations one hop away with their
// matrix elements, sorted by rank.  The Jordan-Wigner string between the two
// sites of a bond gives the fermion sign.
void species_hops(int L, int N, bool periodic, double t, std::vector<uint64_t> &masks,
                  std::vector<uint32_t> &off, std::vector<Hop> &hops) {
    uint64_t n = binom().c[L][N];
    masks.resize(n);
    uint64_t m = (N == 0) ? 0 : ((N == 64) ? ~0ULL : ((1ULL << N) - 1));
    for (uint64_t k = 0; k < n; k++) {
        masks[k] = m;
        if (k + 1 < n) m = next_same_popcount(m);
    }
    off.assign(n + 1, 0);
    hops.clear();
    int nbond = periodic ? L : L - 1;
    std::vector<Hop> tmp;
    for (uint64_t k = 0; k < n; k++) {
        tmp.clear();
        uint64_t s = masks[k];
        if (t != 0.0) {
            for (int b = 0; b < nbond; b++) {
                int i = b, j = (b + 1 == L) ? 0 : b + 1;
                if (((s >> i) ^ (s >> j)) & 1ULL) {
                    int lo = std::min(i, j), hi = std::max(i, j);
                    uint64_t between = (hi - lo > 1) ? (((1ULL << hi) - 1) & ~((2ULL << lo) - 1)) : 0;
                    int par = __builtin_popcountll(s & between) & 1;
                    uint64_t s2 = s ^ (1ULL << i) ^ (1ULL << j);
                    tmp.push_back({(uint32_t)subset_rank(s2), par ? t : -t});
                }
            }
        }
        std::sort(tmp.begin(), tmp.end(), [](const Hop &x, const Hop &y) { return x.rank < y.rank; });
        hops.insert(hops.end(), tmp.begin(), tmp.end());
        off[k + 1] = (uint32_t)hops.size();
    }
}

// Breadth-first labels of the hop graph of one species (reverse
// Cuthill-McKee): a pseudo-peripheral start (repeated breadth-first sweeps
// from the farthest, least-connected configuration), neighbours visited by
// increasing degree and then rank, the visiting order reversed.  Configurations
// one hop apart then get nearby labels, so that the rows a hop connects are
// close in memory.  Disconnected parts are taken in rank order.  Returns
// lab[rank] = label.
std::vector<uint32_t> bfs_labels(const std::vector<uint32_t> &off, const std::vector<Hop> &hops) {
    const int64_t n = (int64_t)off.size() - 1;
    auto deg = [&](int64_t k) { return off[k + 1] - off[k]; };
    std::vector<int64_t> level(n, -1), order;
    order.reserve(n);
    // one sweep from `start` over its component; returns the last level
    auto sweep = [&](int64_t start, std::vector<int64_t> &out) {
        out.clear();
        out.push_back(start);
        level[start] = 0;
        std::vector<std::pair<uint32_t, uint32_t>> nb;
        for (size_t h = 0; h < out.size(); h++) {
            const int64_t k = out[h];
            nb.clear();
            for (uint32_t j = off[k]; j < off[k + 1]; j++)
                if (level[hops[j].rank] < 0) nb.push_back({deg(hops[j].rank), hops[j].rank});
            std::sort(nb.begin(), nb.end());
            for (auto &e : nb)
                if (level[e.second] < 0) {
                    level[e.second] = level[k] + 1;
                    out.push_back(e.second);
                }
        }
        return level[out.back()];
    };
    std::vector<int64_t> comp;
    for (int64_t s0 = 0; s0 < n; s0++) {
        if (level[s0] >= 0) continue;
        int64_t start = s0;
        int64_t ecc = sweep(start, comp);
        for (int round = 0; round < 4; round++) {
            // least-connected configuration of the last level
            int64_t cand = comp.back();
            for (int64_t k : comp)
                if (level[k] == ecc && (deg(k) < deg(cand) || (deg(k) == deg(cand) && k < cand))) cand = k;
            for (int64_t k : comp) level[k] = -1;
            const int64_t e2 = sweep(cand, comp);
            if (e2 <= ecc) {
                if (e2 < ecc) {  // keep the earlier start
                    for (int64_t k : comp) level[k] = -1;
                    sweep(start, comp);
                }
                break;
            }
            start = cand;
            ecc = e2;
        }
        order.insert(order.end(), comp.begin(), comp.end());
    }
    std::vector<uint32_t> lab(n);
    for (int64_t i = 0; i < n; i++) lab[order[i]] = (uint32_t)(n - 1 - i);
    return lab;
}

// Species tables in label order: masks[label], hops of each label with their
// targets as labels, sorted by label.
void relabel_species(const std::vector<uint32_t> &lab, std::vector<uint64_t> &masks, std::vector<uint32_t> &off,
                     std::vector<Hop> &hops) {
    const int64_t n = (int64_t)masks.size();
    std::vector<int64_t> inv(n);
    for (int64_t k = 0; k < n; k++) inv[lab[k]] = k;
    std::vector<uint64_t> m2(n);
    std::vector<uint32_t> o2(n + 1, 0);
    std::vector<Hop> h2;
    h2.reserve(hops.size());
    for (int64_t l = 0; l < n; l++) {
        const int64_t k = inv[l];
        m2[l] = masks[k];
        const size_t b = h2.size();
        for (uint32_t j = off[k]; j < off[k + 1]; j++) h2.push_back({lab[hops[j].rank], hops[j].el});
        std::sort(h2.begin() + b, h2.end(), [](const Hop &x, const Hop &y) { return x.rank < y.rank; });
        o2[l + 1] = (uint32_t)h2.size();
    }
    masks.swap(m2);
    off.swap(o2);
    hops.swap(h2);
}

// One species: configurations, hop lists, in the requested label order
// (0 rank order, 1 breadth-first).
void species(int L, int N, bool periodic, double t, int order, std::vector<uint64_t> &masks,
             std::vector<uint32_t> &off, std::vector<Hop> &hops) {
    species_hops(L, N, periodic, t, masks, off, hops);
    if (order == 1) relabel_species(bfs_labels(off, hops), masks, off, hops);
}

}  // namespace

fd_status build_hubbard(int L, int nup, int ndn, bool periodic, double t, double U, int order, HostCSR &A,
                        std::vector<uint64_t> &cfg_up, std::vector<uint64_t> &cfg_dn) {
    if (L < 3 || L > 62 || nup < 0 || nup > L || ndn < 0 || ndn > L)
        return fail(FD_ERR_INVALID, "Hubbard: need 3 <= L <= 62 and 0 <= n_up, n_dn <= L");
    if (order != 0 && order != 1) return fail(FD_ERR_INVALID, "Hubbard: config_order must be 0 or 1");
    uint64_t nu = binom().c[L][nup], nd = binom().c[L][ndn];
    if (nu * nd >= (1ULL << 32)) return fail(FD_ERR_UNSUPPORTED, "Hubbard: D >= 2^32");
    std::vector<uint64_t> mu, md;
    std::vector<uint32_t> ou, od;
    std::vector<Hop> hu, hd;
    species(L, nup, periodic, t, order, mu, ou, hu);
    species(L, ndn, periodic, t, order, md, od, hd);
    cfg_up = mu;
    cfg_dn = md;
    int64_t D = (int64_t)(nu * nd);
    A.D = D;
    try {
        A.rowptr.assign(D + 1, 0);
    } catch (...) {
        return fail(FD_ERR_OOM, "Hubbard: host allocation");
    }
    for (uint64_t a = 0; a < nu; a++)
        for (uint64_t b = 0; b < nd; b++)
            A.rowptr[a * nd + b + 1] = 1 + (ou[a + 1] - ou[a]) + (od[b + 1] - od[b]);
    for (int64_t i = 0; i < D; i++) A.rowptr[i + 1] += A.rowptr[i];
    int64_t nnz = A.rowptr[D];
    try {
        A.col.resize(nnz);
        A.val.resize(nnz);
    } catch (...) {
        return fail(FD_ERR_OOM, "Hubbard: host allocation");
    }
    parallel_for((int64_t)nu, [&](int64_t a0, int64_t a1) {
        for (int64_t a = a0; a < a1; a++) {
            for (uint64_t b = 0; b < nd; b++) {
                int64_t row = a * (int64_t)nd + b;
                int64_t k = A.rowptr[row];
                const Hop *ub = hu.data() + ou[a], *ue = hu.data() + ou[a + 1];
                const Hop *db = hd.data() + od[b], *de = hd.data() + od[b + 1];
                // up hops into earlier blocks
                for (const Hop *h = ub; h != ue && h->rank < (uint64_t)a; ++h) {
                    A.col[k] = (uint32_t)(h->rank * nd + b);
                    A.val[k++] = h->el;
                }
                // the block of row a: down hops and the diagonal, by column
                bool diag_done = false;
                for (const Hop *h = db; h != de; ++h) {
                    if (!diag_done && h->rank > b) {
                        A.col[k] = (uint32_t)row;
                        A.val[k++] = U * (double)__builtin_popcountll(mu[a] & md[b]);
                        diag_done = true;
                    }
                    A.col[k] = (uint32_t)(a * nd + h->rank);
                    A.val[k++] = h->el;
                }
                if (!diag_done) {
                    A.col[k] = (uint32_t)row;
                    A.val[k++] = U * (double)__builtin_popcountll(mu[a] & md[b]);
                }
                // up hops into later blocks
                for (const Hop *h = ub; h != ue; ++h)
                    if (h->rank > (uint64_t)a) {
                        A.col[k] = (uint32_t)(h->rank * nd + b);
                        A.val[k++] = h->el;
                    }
            }
        }
    });
    return FD_OK;
}

fd_status hubbard_tables(int L, int nup, int ndn, bool periodic, double t, double U, int order, HubbardTables &T) {
    if (L < 3 || L > 62 || nup < 0 || nup > L || ndn < 0 || ndn > L)
        return fail(FD_ERR_INVALID, "Hubbard: need 3 <= L <= 62 and 0 <= n_up, n_dn <= L");
    if (order != 0 && order != 1) return fail(FD_ERR_INVALID, "Hubbard: config_order must be 0 or 1");
    if ((uint64_t)binom().c[L][nup] * binom().c[L][ndn] >= (1ULL << 32))
        return fail(FD_ERR_UNSUPPORTED, "Hubbard: D >= 2^32");
    std::vector<uint32_t> ou, od;
    std::vector<Hop> hu, hd;
    species(L, nup, periodic, t, order, T.mu, ou, hu);
    species(L, ndn, periodic, t, order, T.md, od, hd);
    T.nu = (int64_t)T.mu.size();
    T.nd = (int64_t)T.md.size();
    T.U = U;
    T.off_u.assign(ou.begin(), ou.end());
    T.off_d.assign(od.begin(), od.end());
    for (const Hop &h : hu) {
        T.idx_u.push_back((int32_t)h.rank);
        T.val_u.push_back(h.el);
    }
    for (const Hop &h : hd) {
        T.idx_d.push_back((int32_t)h.rank);
        T.val_d.push_back(h.el);
    }
    return FD_OK;
}

int64_t hubbard_tables_nnz(const HubbardTables &T) {
    return T.nu * T.nd + (int64_t)T.idx_u.size() * T.nd + (int64_t)T.idx_d.size() * T.nu;
}

// Gershgorin interval of the tensor-product form: row (a, b) has centre
// U popcount(mu[a] & md[b]) and radius sum |up hops of a| + sum |down hops of b|.
void hubbard_tables_gershgorin(const HubbardTables &T, double &lo, double &hi) {
    std::vector<double> ru(T.nu, 0.0), rd(T.nd, 0.0);
    for (int64_t a = 0; a < T.nu; a++)
        for (int32_t j = T.off_u[a]; j < T.off_u[a + 1]; j++) ru[a] += std::fabs(T.val_u[j]);
    for (int64_t b = 0; b < T.nd; b++)
        for (int32_t j = T.off_d[b]; j < T.off_d[b + 1]; j++) rd[b] += std::fabs(T.val_d[j]);
    lo = HUGE_VAL;
    hi = -HUGE_VAL;
    for (int64_t a = 0; a < T.nu; a++)
        for (int64_t b = 0; b < T.nd; b++) {
            const double c = T.U * (double)__builtin_popcountll(T.mu[a] & T.md[b]);
            const double r = ru[a] + rd[b];
            lo = std::min(lo, c - r);
            hi = std::max(hi, c + r);
        }
    if (T.nu * T.nd == 0) lo = hi = 0.0;
}

fd_status build_anderson(int L, double t, double W, uint64_t seed, int64_t skip, HostCSR &A) {
    if (L < 3 || (int64_t)L * L * L >= (1LL << 32) || skip < 0)
        return fail(FD_ERR_INVALID, "Anderson: need L >= 3, L^3 < 2^32 and skip >= 0");
    const int64_t L1 = L, L2 = (int64_t)L * L, D = L2 * L;
    A.D = D;
    try {
        A.rowptr.resize(D + 1);
        A.col.resize(7 * D);
        A.val.resize(7 * D);
    } catch (...) {
        return fail(FD_ERR_OOM, "Anderson: host allocation");
    }
    parallel_for(D, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; i++) {
            // SplitMix64 is counter based: the state after i+1 draws is
            // seed + (i+1) * gamma, so row i's disorder needs no sequential pass.
            uint64_t z = seed + (uint64_t)(i + 1 + skip) * 0x9E3779B97F4A7C15ULL;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
            z ^= z >> 31;
            double u = (double)(z >> 11) * 0x1.0p-53;
            int64_t x = i % L1, y = (i / L1) % L1, zz = i / L2;
            int64_t nbr[7] = {i,
                              i - x + (x + 1) % L1, i - x + (x + L1 - 1) % L1,
                              i + L1 * (((y + 1) % L1) - y), i + L1 * (((y + L1 - 1) % L1) - y),
                              i + L2 * (((zz + 1) % L1) - zz), i + L2 * (((zz + L1 - 1) % L1) - zz)};
            std::sort(nbr, nbr + 7);
            A.rowptr[i] = 7 * i;
            for (int p = 0; p < 7; p++) {
                A.col[7 * i + p] = (uint32_t)nbr[p];
                A.val[7 * i + p] = (nbr[p] == i) ? W * (u - 0.5) : -t;
            }
        }
    });
    A.rowptr[D] = 7 * D;
    return FD_OK;
}

fd_status build_diagonal(int64_t n, const double *d, HostCSR &A) {
    if (n < 1 || !d || n >= (1LL << 32)) return fail(FD_ERR_INVALID, "diagonal: need 1 <= n < 2^32 and data");
    A.D = n;
    A.rowptr.resize(n + 1);
    A.col.resize(n);
    A.val.assign(d, d + n);
    for (int64_t i = 0; i <= n; i++) A.rowptr[i] = i;
    for (int64_t i = 0; i < n; i++) A.col[i] = (uint32_t)i;
    return FD_OK;
}

fd_status build_user(int64_t D, const int64_t *rowptr, const uint32_t *col, const double *val,
                     HostCSR &A) {
    if (D < 1 || D >= (1LL << 32) || !rowptr || !col || !val)
        return fail(FD_ERR_INVALID, "user CSR: need 1 <= D < 2^32 and arrays");
    if (rowptr[0] != 0) return fail(FD_ERR_INVALID, "user CSR: rowptr[0] != 0");
    for (int64_t i = 0; i < D; i++) {
        if (rowptr[i + 1] < rowptr[i]) return fail(FD_ERR_INVALID, "user CSR: rowptr decreasing");
        bool has_diag = false;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) {
            if (col[k] >= (uint64_t)D) return fail(FD_ERR_INVALID, "user CSR: column out of range");
            if (k > rowptr[i] && col[k] <= col[k - 1])
                return fail(FD_ERR_INVALID, "user CSR: columns not strictly ascending");
            has_diag |= (col[k] == (uint64_t)i);
        }
        if (!has_diag) return fail(FD_ERR_INVALID, "user CSR: every row must store its diagonal");
    }
    int64_t nnz = rowptr[D];
    A.D = D;
    A.rowptr.assign(rowptr, rowptr + D + 1);
    A.col.assign(col, col + nnz);
    A.val.assign(val, val + nnz);
    return FD_OK;
}

fd_status build_sell(const HostCSR &A, int C, int sigma, HostSELL &S) {
    if (C < 1 || C > 64 || (C & (C - 1)) || sigma < 1)
        return fail(FD_ERR_INVALID, "SELL: C must be a power of two in [1, 64], sigma >= 1");
    const int64_t D = A.D;
    S.C = C;
    S.sigma = sigma;
    S.perm.resize(D);
    std::iota(S.perm.begin(), S.perm.end(), 0);
    auto len = [&](int32_t r) { return A.rowptr[r + 1] - A.rowptr[r]; };
    for (int64_t w = 0; w < D; w += sigma) {
        auto b = S.perm.begin() + w, e = S.perm.begin() + std::min<int64_t>(D, w + sigma);
        std::stable_sort(b, e, [&](int32_t p, int32_t q) { return len(p) > len(q); });
    }
    return fill_sell(A, S);
}

// Chunks of S.C rows in the order S.perm (perm[new] = old), column-major
// inside a chunk, padded to the chunk's longest row.
fd_status fill_sell(const HostCSR &A, HostSELL &S) {
    const int64_t D = A.D;
    const int C = S.C;
    auto len = [&](int32_t r) { return A.rowptr[r + 1] - A.rowptr[r]; };
    int64_t nch = (D + C - 1) / C;
    S.chunk_len.assign(nch, 0);
    S.chunk_ptr.assign(nch + 1, 0);
    for (int64_t s = 0; s < D; s++) {
        int32_t &cl = S.chunk_len[s / C];
        cl = std::max<int32_t>(cl, (int32_t)len(S.perm[s]));
    }
    for (int64_t c = 0; c < nch; c++) S.chunk_ptr[c + 1] = S.chunk_ptr[c] + (int64_t)S.chunk_len[c] * C;
    int64_t total = S.chunk_ptr[nch];
    try {
        S.col.assign(total, 0);
        S.val.assign(total, 0.0);
    } catch (...) {
        return fail(FD_ERR_OOM, "SELL: host allocation");
    }
    parallel_for(nch, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; c++) {
            for (int r = 0; r < C; r++) {
                int64_t s = c * C + r;
                if (s >= D) continue;  // padding slots past D keep column 0, value 0
                int32_t o = S.perm[s];
                int64_t b = A.rowptr[o], n = len(o);
                for (int64_t j = 0; j < S.chunk_len[c]; j++) {
                    int64_t at = S.chunk_ptr[c] + j * C + r;
                    if (j < n) {
                        S.col[at] = A.col[b + j];
                        S.val[at] = A.val[b + j];
                    } else {
                        S.col[at] = (uint32_t)o;
                    }
                }
            }
        }
    });
    return FD_OK;
}

// Walk of the L^3 lattice in pencils: (x, y) tiles of tx by ty sites, tiles
// in x-then-y order, each tile running over all z (z outermost inside the
// tile, then y, then x).  walk[r] = natural index x + L y + L^2 z of the r-th
// site; tiles wider than the lattice cover it whole.
static void tile_walk(int L, int tx, int ty, int32_t *walk) {
    tx = std::min(tx, L);
    ty = std::min(ty, L);
    const int64_t L1 = L, L2 = L1 * L1;
    int64_t r = 0;
    for (int y0 = 0; y0 < L; y0 += ty)
        for (int x0 = 0; x0 < L; x0 += tx)
            for (int64_t z = 0; z < L; z++)
                for (int y = y0; y < std::min(L, y0 + ty); y++)
                    for (int x = x0; x < std::min(L, x0 + tx); x++) walk[r++] = (int32_t)(x + L1 * y + L2 * z);
}

// Pencil order: rows stay the CSR rows (C = 1); only the order in which the
// kernels walk them changes (the row permutation is the tile walk).
fd_status build_pencil(const HostCSR &A, int L, int tx, int ty, HostSELL &S) {
    const int64_t D = A.D;
    if (L < 3 || (int64_t)L * L * L != D || tx < 1 || ty < 1)
        return fail(FD_ERR_INVALID, "pencil order: need the L^3 lattice and tiles of at least one site");
    if (D >= (int64_t(1) << 31)) return fail(FD_ERR_UNSUPPORTED, "pencil order: the walk is indexed in int32");
    S.C = 1;
    S.sigma = 1;
    try {
        S.perm.resize(D);
    } catch (...) {
        return fail(FD_ERR_OOM, "pencil order: host allocation");
    }
    tile_walk(L, tx, ty, S.perm.data());
    return fill_sell(A, S);
}

// Tiled site numbering: the r-th site of the tile walk becomes row r, i.e.
// B = P A P^T with P the walk's permutation (B_rs = A_{walk[r], walk[s]}),
// columns ascending per row.  Same entries, same spectrum; a site's lattice
// neighbours lie within tx ty rows of it except across tile edges.
fd_status relabel_tiles(int L, int tx, int ty, HostCSR &A) {
    const int64_t D = A.D;
    if (L < 3 || (int64_t)L * L * L != D || tx < 1 || ty < 1)
        return fail(FD_ERR_INVALID, "tiled numbering: need the L^3 lattice and tiles of at least one site");
    if (D >= (int64_t(1) << 31)) return fail(FD_ERR_UNSUPPORTED, "tiled numbering: the walk is indexed in int32");
    HostCSR B;
    std::vector<int32_t> walk, inv;
    try {
        walk.resize(D);
        inv.resize(D);
        B.rowptr.resize(D + 1);
        B.col.resize(A.col.size());
        B.val.resize(A.val.size());
    } catch (...) {
        return fail(FD_ERR_OOM, "tiled numbering: host allocation");
    }
    tile_walk(L, tx, ty, walk.data());
    for (int64_t r = 0; r < D; r++) inv[walk[r]] = (int32_t)r;
    B.D = D;
    B.rowptr[0] = 0;
    for (int64_t r = 0; r < D; r++) B.rowptr[r + 1] = B.rowptr[r] + (A.rowptr[walk[r] + 1] - A.rowptr[walk[r]]);
    parallel_for(D, [&](int64_t r0, int64_t r1) {
        std::vector<std::pair<uint32_t, double>> row;
        for (int64_t r = r0; r < r1; r++) {
            const int64_t o = walk[r];
            row.clear();
            for (int64_t k = A.rowptr[o]; k < A.rowptr[o + 1]; k++) row.emplace_back((uint32_t)inv[A.col[k]], A.val[k]);
            std::sort(row.begin(), row.end(),
                      [](const std::pair<uint32_t, double> &a, const std::pair<uint32_t, double> &b) {
                          return a.first < b.first;
                      });
            int64_t k = B.rowptr[r];
            for (const auto &e : row) {
                B.col[k] = e.first;
                B.val[k] = e.second;
                k++;
            }
        }
    });
    A = std::move(B);
    return FD_OK;
}

void gershgorin(const HostCSR &A, double &lo, double &hi) {
    lo = INFINITY;
    hi = -INFINITY;
    for (int64_t i = 0; i < A.D; i++) {
        double c = 0, r = 0;
        for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; k++) {
            if (A.col[k] == (uint64_t)i) c += A.val[k];
            else r += std::fabs(A.val[k]);
        }
        lo = std::min(lo, c - r);
        hi = std::max(hi, c + r);
    }
}

// Window coefficients (Sec. 2: p(x) = sum_k mu_k T_k(x)).  The indicator of
// [a, b] has c_k = (2 - delta_k0)/pi * int_{acos b}^{acos a} cos(k th) dth;
// Jackson damping for M = n + 1 moments multiplies by
// g_k = [(M - k + 1) cos(k q) + sin(k q) cot q] / (M + 1), q = pi / (M + 1).
fd_status cheb_coeffs(int kind, double a, double b, int n, double *mu) {
    if (n < 0 || !mu) return fail(FD_ERR_INVALID, "coefficients: need degree >= 0");
    if (!(a >= -1.0 && a <= 1.0)) return fail(FD_ERR_INVALID, "coefficients: a outside [-1, 1]");
    if ((kind == 0 || kind == 2) && !(b >= a && b <= 1.0)) return fail(FD_ERR_INVALID, "coefficients: need a <= b <= 1");
    if (kind < 0 || kind > 2) return fail(FD_ERR_INVALID, "coefficients: kind must be 0, 1 or 2");
    const double M = n + 1.0, q = M_PI / (M + 1.0), cotq = std::cos(q) / std::sin(q);
    const double tha = std::acos(a), thb = (kind != 1) ? std::acos(b) : 0.0;
    for (int k = 0; k <= n; k++) {
        // kind 2: the indicator's plain coefficients (no damping)
        double g = kind == 2 ? 1.0 : ((M - k + 1.0) * std::cos(k * q) + std::sin(k * q) * cotq) / (M + 1.0);
        double c;
        if (kind != 1)
            c = (k == 0) ? (tha - thb) / M_PI : 2.0 / (k * M_PI) * (std::sin(k * tha) - std::sin(k * thb));
        else
            c = (k == 0 ? 1.0 : 2.0) * std::cos(k * tha);
        mu[k] = g * c;
    }
    return FD_OK;
}

}  // namespace fd
