// Host-side setup: block extraction and validation (Sec. 2) and the shared
// multigrid-reduction hierarchy on A_inn (Sec. 3.2, Alg. 2, eqs. (3.13)-(3.15)).
//
// Pattern-deciding arithmetic (strength thresholds, symbolic products) is
// compiled without floating-point contraction so that each decision is one
// IEEE multiply followed by an exact comparison.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <numeric>
#include <thread>
#include <utility>

#include "internal.hpp"

namespace msp {

// ------------------------------------------------------------------ hashing

uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double unit_centered(uint64_t x) {
    return static_cast<double>(splitmix64(x)) / 18446744073709551616.0 - 0.5;
}

static int popcount_parity(uint32_t x) { return __builtin_popcount(x) & 1; }

// ------------------------------------------------------------------ row-parallel loops

// Threads a row loop may use: at most 16 (MSP_SETUP_THREADS overrides, 1..64);
// inside the per-subsystem workers, their share of that.
static thread_local int t_share = 0;

static int setup_threads() {
    if (t_share > 0) return t_share;
    static const int all = [] {
        const char* v = std::getenv("MSP_SETUP_THREADS");
        const int e = v ? std::atoi(v) : 0;
        if (e > 0) return std::min(e, 64);
        return static_cast<int>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    }();
    return all;
}

// fn(lo, hi, chunk) over contiguous row ranges [lo, hi) covering [0, n), chunk =
// 0 .. chunks-1 in row order; returns the number of chunks.  Every row is
// computed by one thread with the serial loop's arithmetic, so the results do not
// depend on the thread count.  The first exception of any chunk is rethrown.
template <typename F>
static int parallel_rows(int64_t n, F&& fn, int64_t grain = 2048) {
    const int nt = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(setup_threads(), n / grain)));
    if (nt == 1) {
        fn(int64_t(0), n, 0);
        return 1;
    }
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> err(nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            try {
                fn(n * t / nt, n * (t + 1) / nt, t);
            } catch (...) {
                err[t] = std::current_exception();
            }
        });
    for (auto& x : th) x.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
    return nt;
}

// Row pieces of a CSR matrix computed per chunk, then concatenated in row order.
struct CsrPiece {
    std::vector<int64_t> len;
    std::vector<int32_t> ci;
    std::vector<double> v;
};

static void join_pieces(Csr& C, std::vector<CsrPiece>& pc, int chunks) {
    C.rp.assign(C.nr + 1, 0);
    int64_t r = 0, nnz = 0;
    for (int t = 0; t < chunks; ++t) nnz += static_cast<int64_t>(pc[t].ci.size());
    C.ci.clear();
    C.v.clear();
    C.ci.reserve(nnz);
    C.v.reserve(nnz);
    for (int t = 0; t < chunks; ++t) {
        for (int64_t l : pc[t].len) {
            C.rp[r + 1] = C.rp[r] + l;
            ++r;
        }
        C.ci.insert(C.ci.end(), pc[t].ci.begin(), pc[t].ci.end());
        C.v.insert(C.v.end(), pc[t].v.begin(), pc[t].v.end());
        CsrPiece().len.swap(pc[t].len);
    }
}

// ------------------------------------------------------------------ sparse kernels

Csr transpose(const Csr& A) {
    Csr T;
    T.nr = A.nc;
    T.nc = A.nr;
    T.rp.assign(T.nr + 1, 0);
    const int64_t nnz = A.nnz();
    for (int64_t k = 0; k < nnz; ++k) T.rp[A.ci[k] + 1]++;
    for (int64_t i = 0; i < T.nr; ++i) T.rp[i + 1] += T.rp[i];
    T.ci.resize(nnz);
    T.v.resize(nnz);
    std::vector<int64_t> pos(T.rp.begin(), T.rp.end() - 1);
    for (int64_t i = 0; i < A.nr; ++i)
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int64_t p = pos[A.ci[k]]++;
            T.ci[p] = static_cast<int32_t>(i);
            T.v[p] = A.v[k];
        }
    return T;   // rows of T come out sorted because rows of A are visited in order
}

std::vector<int64_t> transpose_map(const Csr& A) {
    const int64_t nnz = A.nnz();
    std::vector<int64_t> rp(A.nc + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) rp[A.ci[k] + 1]++;
    for (int64_t i = 0; i < A.nc; ++i) rp[i + 1] += rp[i];
    std::vector<int64_t> map(nnz);
    for (int64_t i = 0; i < A.nr; ++i)
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) map[rp[A.ci[k]]++] = k;
    return map;
}

std::vector<Csr> interpolation_patterns(const Csr& A, const std::vector<int8_t>& cf, int steps) {
    const int64_t n = A.nr;
    std::vector<int32_t> cnum(n, -1), fnum(n, -1);
    int32_t nc = 0, nf = 0;
    std::vector<int64_t> fidx;
    for (int64_t i = 0; i < n; ++i) {
        if (cf[i]) cnum[i] = nc++;
        else {
            fnum[i] = nf++;
            fidx.push_back(i);
        }
    }
    std::vector<Csr> out;
    for (int t = 0; t < steps; ++t) {
        const Csr* prev = t > 0 ? &out.back() : nullptr;
        Csr W;
        W.nr = nf;
        W.nc = nc;
        std::vector<CsrPiece> pc(64);
        const int chunks = parallel_rows(nf, [&](int64_t lo, int64_t hi, int tc) {
        CsrPiece& piece = pc[tc];
        std::vector<int64_t> mark(nc, -1);
        std::vector<int32_t> cols;
        for (int64_t r = lo; r < hi; ++r) {
            const int64_t i = fidx[r];
            cols.clear();
            for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                const int32_t c = A.ci[k];
                if (c == i) continue;
                if (cf[c]) {
                    if (mark[cnum[c]] != r) {
                        mark[cnum[c]] = r;
                        cols.push_back(cnum[c]);
                    }
                } else if (prev) {
                    const int32_t f = fnum[c];
                    for (int64_t p = prev->rp[f]; p < prev->rp[f + 1]; ++p)
                        if (mark[prev->ci[p]] != r) {
                            mark[prev->ci[p]] = r;
                            cols.push_back(prev->ci[p]);
                        }
                }
            }
            std::sort(cols.begin(), cols.end());
            piece.ci.insert(piece.ci.end(), cols.begin(), cols.end());
            piece.len.push_back(static_cast<int64_t>(cols.size()));
        }
        });
        join_pieces(W, pc, chunks);
        W.v.clear();
        out.push_back(std::move(W));
    }
    return out;
}

Csr spgemm(const Csr& A, const Csr& B) {
    Csr C;
    C.nr = A.nr;
    C.nc = B.nc;
    std::vector<CsrPiece> pc(64);
    const int chunks = parallel_rows(A.nr, [&](int64_t lo, int64_t hi, int t) {
        CsrPiece& out = pc[t];
        std::vector<int64_t> mark(B.nc, -1);
        std::vector<double> acc(B.nc, 0.0);
        std::vector<int32_t> cols;
        for (int64_t i = lo; i < hi; ++i) {
            cols.clear();
            for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                const int32_t j = A.ci[k];
                const double a = A.v[k];
                for (int64_t q = B.rp[j]; q < B.rp[j + 1]; ++q) {
                    const int32_t c = B.ci[q];
                    if (mark[c] != i) {
                        mark[c] = i;
                        acc[c] = 0.0;
                        cols.push_back(c);
                    }
                    acc[c] += a * B.v[q];
                }
            }
            std::sort(cols.begin(), cols.end());
            for (int32_t c : cols) {
                out.ci.push_back(c);
                out.v.push_back(acc[c]);
            }
            out.len.push_back(static_cast<int64_t>(cols.size()));
        }
    });
    join_pieces(C, pc, chunks);
    return C;
}

static void spmv(const Csr& A, const double* x, double* y) {
    parallel_rows(A.nr, [&](int64_t lo, int64_t hi, int) {
        for (int64_t i = lo; i < hi; ++i) {
            double s = 0.0;
            for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) s += A.v[k] * x[A.ci[k]];
            y[i] = s;
        }
    });
}

// ------------------------------------------------------------------ block extraction

// Sorted, zero-free copy of the caller's matrix, checked for valid indices,
// duplicates and exact symmetry; src[k] = position of entry k in the caller's arrays.
static Csr checked_copy(const msp_csr* A, std::vector<int64_t>* src = nullptr) {
    const int64_t n = A->n;
    if (n >= (int64_t(1) << 31)) throw Error(MSP_ERR_UNSUPPORTED, "n must fit in int32");
    const int64_t* rp = A->rowptr;
    if (rp[0] != 0) throw Error(MSP_ERR_ARG, "rowptr[0] must be 0");
    for (int64_t g = 0; g < n; ++g)
        if (rp[g + 1] < rp[g]) throw Error(MSP_ERR_ARG, "rowptr must be non-decreasing");
    const int64_t nnz = rp[n];
    for (int64_t k = 0; k < nnz; ++k)
        if (A->col[k] < 0 || A->col[k] >= n) throw Error(MSP_ERR_ARG, "column index out of range");
    Csr As;
    As.nr = As.nc = n;
    As.rp.assign(n + 1, 0);
    As.ci.reserve(nnz);
    As.v.reserve(nnz);
    std::vector<std::pair<int32_t, int64_t>> row;   // (column, caller position)
    if (src) {
        src->clear();
        src->reserve(nnz);
    }
    for (int64_t g = 0; g < n; ++g) {
        row.clear();
        for (int64_t k = rp[g]; k < rp[g + 1]; ++k)
            if (A->val[k] != 0.0 || std::isnan(A->val[k])) row.emplace_back(A->col[k], k);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, int64_t>& x, const std::pair<int32_t, int64_t>& y) { return x.first < y.first; });
        for (size_t q = 1; q < row.size(); ++q)
            if (row[q].first == row[q - 1].first) throw Error(MSP_ERR_ARG, "duplicate entry in a row");
        for (auto& e : row) {
            As.ci.push_back(e.first);
            As.v.push_back(A->val[e.second]);
            if (src) src->push_back(e.second);
        }
        As.rp[g + 1] = static_cast<int64_t>(As.ci.size());
    }
    // exact symmetry
    for (int64_t g = 0; g < n; ++g)
        for (int64_t k = As.rp[g]; k < As.rp[g + 1]; ++k) {
            const int32_t h = As.ci[k];
            const int32_t* b = As.ci.data() + As.rp[h];
            const int32_t* e = As.ci.data() + As.rp[h + 1];
            const int32_t* f = std::lower_bound(b, e, static_cast<int32_t>(g));
            if (f == e || *f != g || !(As.v[f - As.ci.data()] == As.v[k]))
                throw Error(MSP_ERR_NOT_SYMMETRIC, "matrix is not exactly symmetric");
        }
    return As;
}

SymParts extract_blocks(const msp_csr* A, const msp_symmap* map) {
    if (!A || !map || !A->rowptr || !A->col || !A->val || !map->img)
        throw Error(MSP_ERR_ARG, "null matrix or map");
    if (map->s < 0 || map->s > 6) throw Error(MSP_ERR_ARG, "s must be in 0..6");
    const int s = map->s;
    const int S = 1 << s;
    const int64_t n = A->n;
    if (n <= 0 || map->n_b <= 0 || (map->n_b << s) != n)
        throw Error(MSP_ERR_ARG, "n must equal n_b * 2^s and be positive");
    const int64_t n_b = map->n_b;
    std::vector<int64_t> asrc;
    const Csr As = checked_copy(A, &asrc);

    // map: permutation, inverse
    std::vector<int32_t> inv_i(n, -1);
    std::vector<int8_t> inv_a(n, 0);
    for (int64_t i = 0; i < n_b; ++i)
        for (int a = 0; a < S; ++a) {
            const int64_t g = map->img[i * S + a];
            if (g < 0 || g >= n || inv_i[g] >= 0) throw Error(MSP_ERR_BAD_MAP, "symmetry map is not a permutation");
            inv_i[g] = static_cast<int32_t>(i);
            inv_a[g] = static_cast<int8_t>(a);
        }

    // block structure: row of image a of base cell i, read as (j = a xor b, l)
    SymParts P;
    P.s = s;
    P.n = n;
    P.n_b = n_b;
    P.img.assign(map->img, map->img + n_b * S);
    P.sigma.assign(n_b * S, 0.0);
    P.iface.assign(n_b, 0);
    P.Ainn.nr = P.Ainn.nc = n_b;
    P.Ainn.rp.assign(n_b + 1, 0);
    P.src_nnz = A->rowptr[n];
    P.out_src.assign(static_cast<size_t>(n_b) * (S - 1), -1);
    struct Ent { int32_t j; int32_t l; double v; int64_t src; };
    std::vector<Ent> canon, cur;
    auto row_entries = [&](int64_t g, int a, std::vector<Ent>& out) {
        out.clear();
        for (int64_t k = As.rp[g]; k < As.rp[g + 1]; ++k) {
            const int32_t h = As.ci[k];
            out.push_back({a ^ inv_a[h], inv_i[h], As.v[k], asrc[k]});
        }
        std::sort(out.begin(), out.end(), [](const Ent& x, const Ent& y) {
            return x.j != y.j ? x.j < y.j : x.l < y.l;
        });
    };
    std::vector<double> hdiag(S);
    for (int64_t i = 0; i < n_b; ++i) {
        row_entries(map->img[i * S], 0, canon);
        for (int a = 1; a < S; ++a) {
            row_entries(map->img[i * S + a], a, cur);
            bool same = cur.size() == canon.size();
            for (size_t q = 0; same && q < cur.size(); ++q)
                same = cur[q].j == canon[q].j && cur[q].l == canon[q].l && cur[q].v == canon[q].v;
            if (!same)
                throw Error(MSP_ERR_NOT_SYMMETRIC,
                            "matrix does not have the mirrored block structure of the map");
        }
        std::fill(hdiag.begin(), hdiag.end(), 0.0);
        for (const Ent& e : canon) {
            if (e.j == 0) {
                P.Ainn.ci.push_back(e.l);
                P.Ainn.v.push_back(e.v);
                P.inn_src.push_back(e.src);
            } else {
                if (e.l != i)
                    throw Error(MSP_ERR_UNSUPPORTED,
                                "outer blocks H_j (j != 0) must be diagonal (two-point stencils)");
                hdiag[e.j] = e.v;
                P.out_src[static_cast<size_t>(i) * (S - 1) + (e.j - 1)] = e.src;
                P.iface[i] = 1;
            }
        }
        P.Ainn.rp[i + 1] = static_cast<int64_t>(P.Ainn.ci.size());
        for (int a = 0; a < S; ++a) {
            double acc = 0.0;
            for (int j = 1; j < S; ++j) {
                const double t = popcount_parity(static_cast<uint32_t>(a & j)) ? -hdiag[j] : hdiag[j];
                acc = acc + t;
            }
            P.sigma[i * S + a] = acc;
        }
    }
    return P;
}

// ------------------------------------------------------------------ strength and graphs

struct Graph {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
};

// S_i = {j != i : -a_ij >= theta * max_{l != i} -a_il}, empty if that max <= 0.
static Graph strength(const Csr& A, double theta) {
    Graph S;
    S.rp.assign(A.nr + 1, 0);
    for (int64_t i = 0; i < A.nr; ++i) {
        double mx = -INFINITY;
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (A.ci[k] != i) mx = std::max(mx, -A.v[k]);
        if (mx > 0.0) {
            const double thr = theta * mx;
            for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                if (A.ci[k] != i && -A.v[k] >= thr) S.ci.push_back(A.ci[k]);
        }
        S.rp[i + 1] = static_cast<int64_t>(S.ci.size());
    }
    return S;
}

static Graph symmetrise(const Graph& S, int64_t n) {
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = S.rp[i]; k < S.rp[i + 1]; ++k) {
            cnt[i + 1]++;
            cnt[S.ci[k] + 1]++;
        }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> adj(cnt[n]);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = S.rp[i]; k < S.rp[i + 1]; ++k) {
            adj[pos[i]++] = S.ci[k];
            adj[pos[S.ci[k]]++] = static_cast<int32_t>(i);
        }
    Graph T;
    T.rp.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        auto b = adj.begin() + cnt[i], e = adj.begin() + cnt[i + 1];
        std::sort(b, e);
        auto u = std::unique(b, e);
        T.ci.insert(T.ci.end(), b, u);
        T.rp[i + 1] = static_cast<int64_t>(T.ci.size());
    }
    return T;
}

// Lexicographically-first maximal independent set at distance d in the graph
// T restricted to candidate nodes: scan candidates in the given order and
// take a node when no taken node lies within d hops through candidates.
static std::vector<int8_t> mis_scan(const Graph& T, const std::vector<int8_t>& cand,
                                    const std::vector<int32_t>& order, int d) {
    const int64_t n = static_cast<int64_t>(cand.size());
    std::vector<int8_t> taken(n, 0);
    std::vector<int32_t> stamp(n, -1), frontier, next;
    for (int32_t u : order) {
        bool blocked = false;
        frontier.assign(1, u);
        stamp[u] = u;
        for (int depth = 0; depth < d && !blocked; ++depth) {
            next.clear();
            for (int32_t x : frontier) {
                for (int64_t k = T.rp[x]; k < T.rp[x + 1]; ++k) {
                    const int32_t y = T.ci[k];
                    if (!cand[y] || stamp[y] == u) continue;
                    stamp[y] = u;
                    if (taken[y]) {
                        blocked = true;
                        break;
                    }
                    next.push_back(y);
                }
                if (blocked) break;
            }
            frontier.swap(next);
        }
        if (!blocked) taken[u] = 1;
    }
    return taken;
}

// ------------------------------------------------------------------ interpolation

// Jacobi-truncated ideal interpolation with symbolic patterns and row sums
// rescaled to -sum_{l != i} a_il / a_ii; P = [W; I] in fine-row order with
// coarse unknowns numbered by increasing fine index.  With trunc > 0 each F row
// first drops the weights below trunc * (largest magnitude in the row).
static Csr interpolation(const Csr& A, const std::vector<int8_t>& cf, int steps, double trunc = 0.0) {
    const int64_t n = A.nr;
    std::vector<int32_t> cnum(n, -1), fnum(n, -1);
    int32_t nc = 0, nf = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (cf[i]) cnum[i] = nc++;
        else fnum[i] = nf++;
    }
    std::vector<int64_t> fidx;
    fidx.reserve(nf);
    for (int64_t i = 0; i < n; ++i)
        if (!cf[i]) fidx.push_back(i);
    // W rows over F, columns = coarse numbers
    Csr W;
    W.nr = nf;
    W.nc = nc;
    auto build_step = [&](const Csr* Wprev) {
        Csr Wn;
        Wn.nr = nf;
        Wn.nc = nc;
        std::vector<CsrPiece> pc(64);
        const int chunks = parallel_rows(nf, [&](int64_t lo, int64_t hi, int tc) {
        CsrPiece& piece = pc[tc];
        std::vector<int64_t> mark(nc, -1);
        std::vector<double> acc(nc, 0.0), afc(nc, 0.0);
        std::vector<int8_t> has_afc(nc, 0), has_acc(nc, 0);
        std::vector<int32_t> cols;
        for (int64_t r = lo; r < hi; ++r) {
            const int64_t i = fidx[r];
            cols.clear();
            double dii = 0.0;
            // A_FC entries of the row and O W (Gustavson over ascending f)
            for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                const int32_t c = A.ci[k];
                if (c == i) {
                    dii = A.v[k];
                    continue;
                }
                if (cf[c]) {
                    const int32_t q = cnum[c];
                    if (mark[q] != r) {
                        mark[q] = r;
                        has_afc[q] = has_acc[q] = 0;
                        cols.push_back(q);
                    }
                    afc[q] = A.v[k];
                    has_afc[q] = 1;
                } else if (Wprev) {
                    const int32_t f = fnum[c];
                    const double a = A.v[k];
                    for (int64_t p = Wprev->rp[f]; p < Wprev->rp[f + 1]; ++p) {
                        const int32_t q = Wprev->ci[p];
                        if (mark[q] != r) {
                            mark[q] = r;
                            has_afc[q] = has_acc[q] = 0;
                            cols.push_back(q);
                        }
                        if (!has_acc[q]) {
                            acc[q] = 0.0;
                            has_acc[q] = 1;
                        }
                        acc[q] += a * Wprev->v[p];
                    }
                }
            }
            std::sort(cols.begin(), cols.end());
            const double dinv = 1.0 / dii;
            for (int32_t q : cols) {
                double t;
                if (has_afc[q] && has_acc[q]) t = afc[q] + acc[q];
                else if (has_afc[q]) t = afc[q];
                else t = acc[q];
                piece.ci.push_back(q);
                piece.v.push_back(-(dinv * t));
            }
            piece.len.push_back(static_cast<int64_t>(cols.size()));
        }
        });
        join_pieces(Wn, pc, chunks);
        return Wn;
    };
    W = build_step(nullptr);
    for (int t = 1; t < steps; ++t) {
        Csr Wn = build_step(&W);
        W.rp.swap(Wn.rp);
        W.ci.swap(Wn.ci);
        W.v.swap(Wn.v);
    }
    if (trunc > 0.0) {
        Csr T;
        T.nr = nf;
        T.nc = nc;
        T.rp.assign(nf + 1, 0);
        for (int32_t r = 0; r < nf; ++r) {
            double mx = 0.0;
            for (int64_t p = W.rp[r]; p < W.rp[r + 1]; ++p) mx = std::max(mx, std::fabs(W.v[p]));
            const double lim = trunc * mx;
            for (int64_t p = W.rp[r]; p < W.rp[r + 1]; ++p)
                if (std::fabs(W.v[p]) >= lim) {
                    T.ci.push_back(W.ci[p]);
                    T.v.push_back(W.v[p]);
                }
            T.rp[r + 1] = static_cast<int64_t>(T.ci.size());
        }
        W.rp.swap(T.rp);
        W.ci.swap(T.ci);
        W.v.swap(T.v);
    }
    // rescale rows to rho_i = -sum_{l != i} a_il / a_ii
    for (int32_t r = 0; r < nf; ++r) {
        const int64_t i = fidx[r];
        double off = 0.0, dii = 0.0;
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            if (A.ci[k] == i) dii = A.v[k];
            else off += A.v[k];
        }
        const double rho = -off / dii;
        double ws = 0.0;
        for (int64_t p = W.rp[r]; p < W.rp[r + 1]; ++p) ws += W.v[p];
        if (ws != 0.0) {
            const double sc = rho / ws;
            for (int64_t p = W.rp[r]; p < W.rp[r + 1]; ++p) W.v[p] = W.v[p] * sc;
        }
    }
    Csr P;
    P.nr = n;
    P.nc = nc;
    P.rp.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        if (cf[i]) {
            P.ci.push_back(cnum[i]);
            P.v.push_back(1.0);
        } else {
            const int32_t r = fnum[i];
            for (int64_t p = W.rp[r]; p < W.rp[r + 1]; ++p) {
                P.ci.push_back(W.ci[p]);
                P.v.push_back(W.v[p]);
            }
        }
        P.rp[i + 1] = static_cast<int64_t>(P.ci.size());
    }
    return P;
}

// ------------------------------------------------------------------ FSAI and damping

// Dense Cholesky of an SPD k x k row-major matrix in place (lower factor).
static bool cholesky(int k, double* M) {
    for (int j = 0; j < k; ++j) {
        double d = M[j * k + j];
        for (int p = 0; p < j; ++p) d -= M[j * k + p] * M[j * k + p];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        M[j * k + j] = d;
        for (int i = j + 1; i < k; ++i) {
            double s = M[i * k + j];
            for (int p = 0; p < j; ++p) s -= M[i * k + p] * M[j * k + p];
            M[i * k + j] = s / d;
        }
    }
    return true;
}

static double lookup(const Csr& A, int64_t i, int32_t j) {
    const int32_t* b = A.ci.data() + A.rp[i];
    const int32_t* e = A.ci.data() + A.rp[i + 1];
    const int32_t* f = std::lower_bound(b, e, j);
    return (f != e && *f == j) ? A.v[f - A.ci.data()] : 0.0;
}

// Static-pattern FSAI: row i pattern = given lower neighbours (ascending) + i;
// A[J,J] g = e_last solved by Cholesky, g scaled by 1/sqrt(g_last).
static Csr fsai_rows(const Csr& A, const std::vector<std::vector<int32_t>>& lower) {
    Csr G;
    G.nr = G.nc = A.nr;
    std::vector<CsrPiece> pc(64);
    const int chunks = parallel_rows(A.nr, [&](int64_t lo, int64_t hi, int t) {
    CsrPiece& out = pc[t];
    std::vector<double> M, g;
    std::vector<int32_t> J;
    for (int64_t i = lo; i < hi; ++i) {
        J = lower[i];
        J.push_back(static_cast<int32_t>(i));
        const int k = static_cast<int>(J.size());
        M.assign(static_cast<size_t>(k) * k, 0.0);
        for (int p = 0; p < k; ++p)
            for (int q = 0; q < k; ++q) M[p * k + q] = lookup(A, J[p], J[q]);
        if (!cholesky(k, M.data())) throw Error(MSP_ERR_NOT_SPD, "FSAI: local matrix not SPD");
        // solve L L^T g = e_last: L y = e_last has y = e_last / L_kk, then L^T g = y
        g.assign(k, 0.0);
        g[k - 1] = 1.0 / M[(k - 1) * k + (k - 1)];
        for (int p = k - 1; p >= 0; --p) {
            double s = g[p];
            for (int q = p + 1; q < k; ++q) s -= M[q * k + p] * g[q];
            g[p] = s / M[p * k + p];
        }
        const double sc = 1.0 / std::sqrt(g[k - 1]);
        for (int p = 0; p < k; ++p) {
            out.ci.push_back(J[p]);
            out.v.push_back(g[p] * sc);
        }
        out.len.push_back(k);
    }
    }, 256);
    join_pieces(G, pc, chunks);
    return G;
}

Csr fsai_full_lower(const Csr& A) {
    std::vector<std::vector<int32_t>> lower(A.nr);
    for (int64_t i = 0; i < A.nr; ++i)
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (A.ci[k] < i) lower[i].push_back(A.ci[k]);
    return fsai_rows(A, lower);
}

// Adaptive FSAI pattern: row i grows from {i}.  Each step takes the row g
// (g_i = 1, support P) minimising g^T A g, forms r = A g over the rows of P in
// the order they joined (columns ascending within a row), and adds the
// candidate j < i outside P (same block if `block`) with the largest
// r_j^2 / a_jj; scores within kAfsaiTie of the best tie to the smaller column.
// Stops at nnz_max entries or when no score is positive.  Returns the lower
// neighbours of each row, ascending (the diagonal not included).
static constexpr double kAfsaiTie = 1e-10;

static std::vector<std::vector<int32_t>> afsai_lower(const Csr& A, const std::vector<int8_t>* block, int nnz_max) {
    const int64_t n = A.nr;
    std::vector<double> d(n);
    for (int64_t i = 0; i < n; ++i) d[i] = lookup(A, i, static_cast<int32_t>(i));
    std::vector<std::vector<int32_t>> lower(n);
    parallel_rows(n, [&](int64_t lo, int64_t hi, int) {
    std::vector<int64_t> stamp(n, -1);
    std::vector<double> acc(n, 0.0);
    std::vector<int32_t> P, cand;
    std::vector<double> g, M, y;
    int64_t tick = 0;
    for (int64_t i = lo; i < hi; ++i) {
        P.assign(1, static_cast<int32_t>(i));
        g.assign(1, 1.0);
        while (static_cast<int>(P.size()) < nnz_max) {
            ++tick;
            cand.clear();
            for (size_t t = 0; t < P.size(); ++t) {
                const int32_t p = P[t];
                for (int64_t k = A.rp[p]; k < A.rp[p + 1]; ++k) {
                    const int32_t j = A.ci[k];
                    if (j >= i) break;   // columns ascending
                    if (block && (*block)[j] != (*block)[i]) continue;
                    if (std::find(P.begin(), P.end(), j) != P.end()) continue;
                    if (stamp[j] != tick) {
                        stamp[j] = tick;
                        acc[j] = 0.0;
                        cand.push_back(j);
                    }
                    acc[j] += A.v[k] * g[t];
                }
            }
            if (cand.empty()) break;
            double best = 0.0;
            for (int32_t j : cand) best = std::max(best, acc[j] * acc[j] / d[j]);
            if (!(best > 0.0)) break;
            int32_t pick = -1;
            for (int32_t j : cand)
                if (acc[j] * acc[j] / d[j] >= best * (1.0 - kAfsaiTie) && (pick < 0 || j < pick)) pick = j;
            P.push_back(pick);
            // re-minimise: A[Q,Q] y = -A[Q,i], Q = P without i
            const int q = static_cast<int>(P.size()) - 1;
            M.assign(static_cast<size_t>(q) * q, 0.0);
            y.assign(q, 0.0);
            for (int a = 0; a < q; ++a) {
                for (int b = 0; b < q; ++b) M[a * q + b] = lookup(A, P[a + 1], P[b + 1]);
                y[a] = -lookup(A, P[a + 1], static_cast<int32_t>(i));
            }
            if (!cholesky(q, M.data())) throw Error(MSP_ERR_NOT_SPD, "adaptive FSAI: local matrix not SPD");
            for (int a = 0; a < q; ++a) {   // L z = y, then L^T y = z
                double s = y[a];
                for (int b = 0; b < a; ++b) s -= M[a * q + b] * y[b];
                y[a] = s / M[a * q + a];
            }
            for (int a = q - 1; a >= 0; --a) {
                double s = y[a];
                for (int b = a + 1; b < q; ++b) s -= M[b * q + a] * y[b];
                y[a] = s / M[a * q + a];
            }
            g.assign(1, 1.0);
            g.insert(g.end(), y.begin(), y.end());
        }
        lower[i].assign(P.begin() + 1, P.end());
        std::sort(lower[i].begin(), lower[i].end());
    }
    }, 256);
    return lower;
}

// Energy-minimising interpolation: the F rows W of P = [W; I] minimise
// tr(P^T A P) on W's pattern with every row sum of W kept, by `steps`
// conjugate-gradient steps from W.  Half gradient A_FF W + A_FC on the
// pattern; projection onto the constraint's tangent space subtracts each
// row's mean over its pattern; preconditioner: row f divided by a_ff.
static void emin(const Csr& A, const std::vector<int8_t>& cf, Csr& P, int steps) {
    const int64_t n = A.nr;
    std::vector<int32_t> fnum(n, -1), cnum(n, -1), fidx;
    int32_t nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (cf[i]) cnum[i] = nc++;
        else {
            fnum[i] = static_cast<int32_t>(fidx.size());
            fidx.push_back(static_cast<int32_t>(i));
        }
    }
    const int64_t nf = static_cast<int64_t>(fidx.size());
    // W: the F rows of P (entry positions of P kept in wpos)
    std::vector<int64_t> wrp(nf + 1, 0), wpos;
    std::vector<int32_t> wc;
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t i = fidx[f];
        for (int64_t k = P.rp[i]; k < P.rp[i + 1]; ++k) {
            wc.push_back(P.ci[k]);
            wpos.push_back(k);
        }
        wrp[f + 1] = static_cast<int64_t>(wc.size());
    }
    const int64_t m = wrp[nf];
    std::vector<double> w(m), dinv(m);
    for (int64_t e = 0; e < m; ++e) w[e] = P.v[wpos[e]];
    for (int64_t f = 0; f < nf; ++f) {
        const double dd = 1.0 / lookup(A, fidx[f], fidx[f]);
        for (int64_t e = wrp[f]; e < wrp[f + 1]; ++e) dinv[e] = dd;
    }
    // out = A_FF x (+ A_FC if add_afc) on W's pattern, x on W's pattern
    auto apply = [&](const std::vector<double>& x, bool add_afc, std::vector<double>& out) {
        std::vector<double> prod(m, 0.0);
        parallel_rows(nf, [&](int64_t lo, int64_t hi, int) {
        // slot of column c in row f of W (-1: off the pattern), through a dense row map
        std::vector<int64_t> slot(nc, -1);
        for (int64_t f = lo; f < hi; ++f) {
            for (int64_t e = wrp[f]; e < wrp[f + 1]; ++e) slot[wc[e]] = e;
            const int32_t i = fidx[f];
            for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                const int32_t g = fnum[A.ci[k]];
                if (g < 0) continue;
                const double a = A.v[k];
                for (int64_t e = wrp[g]; e < wrp[g + 1]; ++e) {
                    const int64_t q = slot[wc[e]];
                    if (q >= 0) prod[q] += a * x[e];
                }
            }
            for (int64_t e = wrp[f]; e < wrp[f + 1]; ++e) {
                double v = prod[e];
                if (add_afc) {
                    // A_FC entry (f, c): the coupling of fine row i to the coarse point numbered c
                    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                        if (cnum[A.ci[k]] == wc[e]) {
                            v = v + A.v[k];
                            break;
                        }
                }
                out[e] = v;
            }
            for (int64_t e = wrp[f]; e < wrp[f + 1]; ++e) slot[wc[e]] = -1;
        }
        }, 64);
    };
    auto project = [&](std::vector<double>& v) {
        for (int64_t f = 0; f < nf; ++f) {
            const int64_t c = wrp[f + 1] - wrp[f];
            if (c == 0) continue;
            double s = 0.0;
            for (int64_t e = wrp[f]; e < wrp[f + 1]; ++e) s += v[e];
            const double mean = s / static_cast<double>(c);
            for (int64_t e = wrp[f]; e < wrp[f + 1]; ++e) v[e] = v[e] - mean;
        }
    };
    auto dot = [&](const std::vector<double>& a, const std::vector<double>& b) {
        double s = 0.0;
        for (int64_t e = 0; e < m; ++e) s += a[e] * b[e];
        return s;
    };
    std::vector<double> r(m), z(m), p(m), q(m);
    apply(w, true, r);
    project(r);
    for (auto& x : r) x = -x;
    for (int64_t e = 0; e < m; ++e) z[e] = dinv[e] * r[e];
    p = z;
    double rz = dot(r, z);
    for (int it = 0; it < steps; ++it) {
        if (!(rz > 0.0)) break;
        apply(p, false, q);
        project(q);
        const double pq = dot(p, q);
        if (!(pq > 0.0)) break;
        const double alpha = rz / pq;
        for (int64_t e = 0; e < m; ++e) {
            w[e] = w[e] + alpha * p[e];
            r[e] = r[e] - alpha * q[e];
        }
        for (int64_t e = 0; e < m; ++e) z[e] = dinv[e] * r[e];
        const double rz_new = dot(r, z);
        const double beta = rz_new / rz;
        for (int64_t e = 0; e < m; ++e) p[e] = z[e] + beta * p[e];
        rz = rz_new;
    }
    for (int64_t e = 0; e < m; ++e) P.v[wpos[e]] = w[e];
}

// omega = 4 / (3 lam), lam = v^T G A G^T v after 20 power iterations from
// v_i = splitmix64(seed xor i)/2^64 - 1/2 (normalised).
double damping(const Csr& A, const Csr& G, const Csr& GT, uint64_t seed) {
    const int64_t n = A.nr;
    std::vector<double> v(n), t1(n), t2(n), w(n);
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        v[i] = unit_centered(seed ^ static_cast<uint64_t>(i));
        nrm += v[i] * v[i];
    }
    nrm = std::sqrt(nrm);
    for (auto& x : v) x /= nrm;
    double lam = 0.0;
    for (int it = 0; it < 20; ++it) {
        spmv(GT, v.data(), t1.data());
        spmv(A, t1.data(), t2.data());
        spmv(G, t2.data(), w.data());
        double vw = 0.0, ww = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            vw += v[i] * w[i];
            ww += w[i] * w[i];
        }
        lam = vw;
        const double wn = std::sqrt(ww);
        for (int64_t i = 0; i < n; ++i) v[i] = w[i] / wn;
    }
    return 4.0 / (3.0 * lam);
}

// ------------------------------------------------------------------ dense eigen (Jacobi)

void sym_eig(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
    V.assign(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double app = A[p * n + p], aqq = A[q * n + q];
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return A[x * n + x] < A[y * n + y]; });
    w.resize(n);
    std::vector<double> Vs(static_cast<size_t>(n) * n);
    for (int c = 0; c < n; ++c) {
        w[c] = A[idx[c] * n + idx[c]];
        for (int k = 0; k < n; ++k) Vs[k * n + c] = V[k * n + idx[c]];
    }
    V.swap(Vs);
}

// ------------------------------------------------------------------ hierarchy

// Dense inverse of a small SPD matrix: Cholesky A = L L^T, then Linv = L^{-1}
// column by column and A^{-1} = Linv^T Linv (threads over columns).
static std::vector<double> dense_inverse(const Csr& Ac) {
    const int64_t nc = Ac.nr;
    if (nc > 8192) throw Error(MSP_ERR_UNSUPPORTED, "coarsest level too large for a dense solve");
    std::vector<double> M(nc * nc, 0.0);
    for (int64_t i = 0; i < nc; ++i)
        for (int64_t k = Ac.rp[i]; k < Ac.rp[i + 1]; ++k) M[i * nc + Ac.ci[k]] = Ac.v[k];
    if (!cholesky(static_cast<int>(nc), M.data())) throw Error(MSP_ERR_NOT_SPD, "coarsest level is not SPD");
    std::vector<int64_t> coff(nc + 1, 0);
    for (int64_t c = 0; c < nc; ++c) coff[c + 1] = coff[c] + (nc - c);
    std::vector<double> Li(coff[nc]);
    const unsigned nth = static_cast<unsigned>(setup_threads());
    auto parallel = [&](auto&& body) {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nth; ++t)
            th.emplace_back([&, t]() {
                for (int64_t c = t; c < nc; c += nth) body(c);
            });
        for (auto& x : th) x.join();
    };
    parallel([&](int64_t c) {
        double* y = Li.data() + coff[c];   // y[i - c] = Linv[i][c], i >= c
        for (int64_t i = c; i < nc; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            const double* Lr = M.data() + i * nc;
            for (int64_t p = c; p < i; ++p) s -= Lr[p] * y[p - c];
            y[i - c] = s / Lr[i];
        }
    });
    std::vector<double> inv(nc * nc, 0.0);
    parallel([&](int64_t i) {
        const double* ci = Li.data() + coff[i];
        for (int64_t j = i; j < nc; ++j) {
            const double* cj = Li.data() + coff[j];
            double s = 0.0;
            for (int64_t p = j; p < nc; ++p) s += ci[p - i] * cj[p - j];
            inv[i * nc + j] = s;
            inv[j * nc + i] = s;
        }
    });
    return inv;
}

// ------------------------------------------------------------------ domains made of copies

CopyParts extract_copies(const msp_csr* A, const msp_copies* map, const msp_opts& o) {
    if (!A || !map || !A->rowptr || !A->col || !A->val || !map->sub)
        throw Error(MSP_ERR_ARG, "null matrix or copy map");
    const int64_t n = A->n, n_b = map->n_b;
    const int64_t nc = map->copies;
    if (n <= 0 || n_b <= 0 || nc <= 0 || n_b * nc != n)
        throw Error(MSP_ERR_ARG, "n must equal n_b * copies and be positive");
    CopyParts P;
    P.sym.s = 0;
    P.sym.n = P.sym.n_b = n;
    P.sym.Ainn = checked_copy(A, &P.sym.inn_src);
    P.sym.src_nnz = A->rowptr[n];
    const Csr& As = P.sym.Ainn;
    std::vector<int32_t> copy_of(n, -1), base_of(n, -1);
    for (int64_t i = 0; i < n_b; ++i)
        for (int64_t a = 0; a < nc; ++a) {
            const int64_t g = map->sub[i * nc + a];
            if (g < 0 || g >= n || copy_of[g] >= 0) throw Error(MSP_ERR_BAD_MAP, "copy map is not a permutation");
            copy_of[g] = static_cast<int32_t>(a);
            base_of[g] = static_cast<int32_t>(i);
        }
    // Interface (Sec. 3, eq. (3.1)): a base unknown coupled to another copy in
    // some copy, or whose row inside its copy (read in base numbering) differs
    // from the base copy's row in pattern or value.
    P.iface_base.assign(n_b, 0);
    P.A00.nr = P.A00.nc = n_b;
    P.A00.rp.assign(n_b + 1, 0);
    std::vector<std::pair<int32_t, double>> row0, row;
    auto copy_row = [&](int64_t i, int64_t a, std::vector<std::pair<int32_t, double>>& out) {
        out.clear();
        bool cross = false;
        const int64_t g = map->sub[i * nc + a];
        for (int64_t k = As.rp[g]; k < As.rp[g + 1]; ++k) {
            const int32_t h = As.ci[k];
            if (copy_of[h] != a)
                cross = true;
            else
                out.emplace_back(base_of[h], As.v[k]);
        }
        std::sort(out.begin(), out.end(), [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
            return x.first < y.first;
        });
        return cross;
    };
    for (int64_t i = 0; i < n_b; ++i) {
        bool on = copy_row(i, 0, row0);
        for (const auto& e : row0) {
            P.A00.ci.push_back(e.first);
            P.A00.v.push_back(e.second);
        }
        P.A00.rp[i + 1] = static_cast<int64_t>(P.A00.ci.size());
        for (int64_t a = 1; a < nc && !on; ++a) {
            on = copy_row(i, a, row);
            if (!on && row != row0) on = true;
        }
        P.iface_base[i] = on ? 1 : 0;
    }
    // Alg. 2 on the base copy, the split replicated to every copy
    const std::vector<int8_t> cf_base = reduction_split(P.A00, P.iface_base, o);
    P.cf0.assign(n, 0);
    P.sym.iface.assign(n, 0);
    for (int64_t i = 0; i < n_b; ++i)
        for (int64_t a = 0; a < nc; ++a) {
            const int64_t g = map->sub[i * nc + a];
            P.cf0[g] = cf_base[i];
            P.sym.iface[g] = P.iface_base[i];
        }
    P.sym.sigma.assign(n, 0.0);
    P.sym.img.resize(n);
    std::iota(P.sym.img.begin(), P.sym.img.end(), int64_t(0));
    return P;
}

// Alg. 2: the maximal independent set of T^d over the inner nodes, scanned in
// decreasing hash priority of the node index, joined with the interface.
static std::vector<int8_t> reduction_split(const Graph& S, int64_t n, const std::vector<int8_t>& iface,
                                           const msp_opts& o) {
    const Graph T = symmetrise(S, n);
    std::vector<int8_t> cand(n, 1);
    std::vector<int32_t> order;
    for (int64_t i = 0; i < n; ++i) {
        cand[i] = iface[i] ? 0 : 1;
        if (cand[i]) order.push_back(static_cast<int32_t>(i));
    }
    std::vector<uint64_t> pri(n);
    for (int64_t i = 0; i < n; ++i) pri[i] = splitmix64(o.seed ^ static_cast<uint64_t>(i));
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return pri[x] > pri[y]; });
    std::vector<int8_t> cf = mis_scan(T, cand, order, o.dist);
    for (int64_t i = 0; i < n; ++i) cf[i] = (cf[i] || iface[i]) ? 1 : 0;
    return cf;
}

std::vector<int8_t> reduction_split(const Csr& A, const std::vector<int8_t>& iface, const msp_opts& o) {
    return reduction_split(strength(A, o.theta), A.nr, iface, o);
}

// Levels from `lev` down, appended to H, starting from the operator A of that level.
static void build_levels(HostHierarchy& H, Csr A, int lev, const std::vector<int8_t>& iface, const msp_opts& o,
                         const std::vector<int8_t>* cf0) {
    const uint64_t seed = o.seed;
    // MSP_SETUP_LOG set (non-empty, not "0"): seconds per setup phase and level to stderr
    const char* logv = std::getenv("MSP_SETUP_LOG");
    const bool log = logv && *logv && std::strcmp(logv, "0") != 0;
    auto clk = std::chrono::steady_clock::now();
    auto lap = [&](const char* what, int l) {
        if (!log) return;
        const auto t = std::chrono::steady_clock::now();
        std::fprintf(stderr, "msp setup: level %d %s %.3f s\n", l, what, std::chrono::duration<double>(t - clk).count());
        clk = t;
    };
    while (true) {
        H.lev.emplace_back();
        HostLevel& L = H.lev.back();
        const int64_t n = A.nr;
        if (n <= o.coarse_max || lev == o.max_levels - 1) {
            L.A = std::move(A);
            break;
        }
        Graph S = strength(A, o.theta);
        std::vector<int8_t> cf;
        if (lev == 0 && cf0) {
            // a split computed elsewhere (the populated interface of a domain of copies)
            if (static_cast<int64_t>(cf0->size()) != n) throw Error(MSP_ERR_ARG, "level-0 split size");
            cf = *cf0;
        } else if (lev == 0) {
            cf = reduction_split(S, n, iface, o);
        } else {
            // standard level: MIS of T, priority (number of strong dependants, hash)
            Graph T = symmetrise(S, n);
            std::vector<int64_t> lam(n, 0);
            for (int64_t k = 0; k < S.rp[n]; ++k) lam[S.ci[k]]++;
            std::vector<uint64_t> h(n);
            for (int64_t i = 0; i < n; ++i)
                h[i] = splitmix64(seed ^ (static_cast<uint64_t>(lev) << 40) ^ static_cast<uint64_t>(i));
            std::vector<int32_t> order(n);
            std::iota(order.begin(), order.end(), 0);
            std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
                return lam[x] != lam[y] ? lam[x] > lam[y] : h[x] > h[y];
            });
            cf = mis_scan(T, std::vector<int8_t>(n, 1), order, 1);
        }
        lap("split", lev);
        int64_t nc = 0;
        for (int64_t i = 0; i < n; ++i) nc += cf[i];
        if (nc == 0 || static_cast<double>(nc) > o.max_ratio * static_cast<double>(n)) {
            L.A = std::move(A);
            break;
        }
        // smoother: FSAI on the strong lower pattern (or an adaptive one), block-diagonal
        // F/C at level 0
        std::vector<std::vector<int32_t>> lower(n);
        if (o.afsai_nnz > 0) {
            lower = afsai_lower(A, lev == 0 ? &cf : nullptr, o.afsai_nnz);
        } else {
            for (int64_t i = 0; i < n; ++i)
                for (int64_t k = S.rp[i]; k < S.rp[i + 1]; ++k) {
                    const int32_t j = S.ci[k];
                    if (j < i && (lev != 0 || cf[j] == cf[i])) lower[i].push_back(j);
                }
        }
        lap("smoother pattern", lev);
        L.G = fsai_rows(A, lower);
        L.GT = transpose(L.G);
        lap("fsai", lev);
        L.omega = damping(A, L.G, L.GT, seed);
        L.M = spgemm(L.GT, L.G);
        for (double& v : L.M.v) v *= L.omega;
        lap("damping and M", lev);
        L.P = interpolation(A, cf, lev == 0 ? o.jacobi0 : o.jacobi, lev == 0 ? o.trunc0 : 0.0);
        lap("interpolation", lev);
        if (o.emin_steps > 0) emin(A, cf, L.P, o.emin_steps);
        lap("energy minimisation", lev);
        L.R = transpose(L.P);
        L.cf = std::move(cf);
        Csr AP = spgemm(A, L.P);
        Csr Ac = spgemm(L.R, AP);
        lap("galerkin", lev);
        L.A = std::move(A);
        A = std::move(Ac);
        ++lev;
    }
    H.coarse_inv = dense_inverse(H.lev.back().A);
}

HostHierarchy build_hierarchy(const Csr& Ainn, const std::vector<int8_t>& iface, const msp_opts& o,
                              const std::vector<int8_t>* cf0) {
    HostHierarchy H;
    build_levels(H, Ainn, 0, iface, o, cf0);
    return H;
}

HostHierarchy build_hierarchy_below(const HostHierarchy& old, const msp_opts& o) {
    if (old.lev.size() < 2) throw Error(MSP_ERR_ARG, "no level below the reduction level");
    HostHierarchy H;
    H.lev.push_back(old.lev[0]);
    build_levels(H, old.lev[1].A, 1, std::vector<int8_t>(), o, nullptr);
    return H;
}

static bool same_pattern(const Csr& X, const Csr& Y) { return X.rp == Y.rp && X.ci == Y.ci; }

// ------------------------------------------------------------------ AMGS (Sec. 3.1)

// Rows of M without the off-diagonal entries |m_ij| < tau sqrt(|m_ii m_jj|).
static std::vector<std::vector<int32_t>> filtered_rows(const Csr& M, double tau) {
    std::vector<double> d(M.nr, 0.0);
    for (int64_t i = 0; i < M.nr; ++i)
        for (int64_t k = M.rp[i]; k < M.rp[i + 1]; ++k)
            if (M.ci[k] == i) d[i] = std::fabs(M.v[k]);
    std::vector<std::vector<int32_t>> rows(M.nr);
    for (int64_t i = 0; i < M.nr; ++i)
        for (int64_t k = M.rp[i]; k < M.rp[i + 1]; ++k) {
            const int32_t j = M.ci[k];
            if (j == i || std::fabs(M.v[k]) >= tau * std::sqrt(d[i] * d[j])) rows[i].push_back(j);
        }
    return rows;
}

// FSAI of M on the lower triangle of the pattern of M_f^power (power >= 1):
// the cells reachable from row i in at most `power` steps of the filtered graph.
static Csr fsai_filtered_power(const Csr& M, double tau, int power) {
    const std::vector<std::vector<int32_t>> P = filtered_rows(M, tau);
    std::vector<std::vector<int32_t>> lower(M.nr);
    std::vector<int64_t> mark(M.nr, -1);
    std::vector<int32_t> front, next, reach;
    for (int64_t i = 0; i < M.nr; ++i) {
        reach.clear();
        front.assign(1, static_cast<int32_t>(i));
        mark[i] = i;
        for (int step = 0; step < power; ++step) {
            next.clear();
            for (int32_t j : front)
                for (int32_t l : P[j])
                    if (mark[l] != i) {
                        mark[l] = i;
                        next.push_back(l);
                        reach.push_back(l);
                    }
            front.swap(next);
        }
        for (int32_t l : reach)
            if (l < i) lower[i].push_back(l);
        std::sort(lower[i].begin(), lower[i].end());
    }
    return fsai_rows(M, lower);
}

// a X + b Y on the union pattern (rows sorted); sums that are exactly zero are dropped.
static Csr add_csr(const Csr& X, double a, const Csr& Y, double b) {
    Csr Z;
    Z.nr = X.nr;
    Z.nc = X.nc;
    Z.rp.assign(Z.nr + 1, 0);
    for (int64_t i = 0; i < X.nr; ++i) {
        int64_t p = X.rp[i], q = Y.rp[i];
        const int64_t pe = X.rp[i + 1], qe = Y.rp[i + 1];
        while (p < pe || q < qe) {
            int32_t j;
            double v;
            if (q >= qe || (p < pe && X.ci[p] < Y.ci[q])) {
                j = X.ci[p];
                v = a * X.v[p++];
            } else if (p >= pe || Y.ci[q] < X.ci[p]) {
                j = Y.ci[q];
                v = b * Y.v[q++];
            } else {
                j = X.ci[p];
                v = a * X.v[p++] + b * Y.v[q++];
            }
            if (v != 0.0) {
                Z.ci.push_back(j);
                Z.v.push_back(v);
            }
        }
        Z.rp[i + 1] = static_cast<int64_t>(Z.ci.size());
    }
    return Z;
}

// Rows [r0, r1) and columns [c0, c1) of A, columns shifted by c0.
static Csr block_of(const Csr& A, int64_t r0, int64_t r1, int64_t c0, int64_t c1) {
    Csr M;
    M.nr = r1 - r0;
    M.nc = c1 - c0;
    M.rp.assign(M.nr + 1, 0);
    for (int64_t i = r0; i < r1; ++i) {
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (A.ci[k] >= c0 && A.ci[k] < c1) {
                M.ci.push_back(static_cast<int32_t>(A.ci[k] - c0));
                M.v.push_back(A.v[k]);
            }
        M.rp[i - r0 + 1] = static_cast<int64_t>(M.ci.size());
    }
    return M;
}

AmgsParts build_amgs(SymParts& sym, const msp_opts& o) {
    const int64_t nb = sym.n_b;
    const int S = 1 << sym.s;
    // inner cells first, interface cells after, each in increasing base index
    std::vector<int64_t> perm;
    perm.reserve(nb);
    for (int64_t i = 0; i < nb; ++i)
        if (!sym.iface[i]) perm.push_back(i);
    const int64_t nI = static_cast<int64_t>(perm.size());
    for (int64_t i = 0; i < nb; ++i)
        if (sym.iface[i]) perm.push_back(i);
    if (nI == 0 || nI == nb) throw Error(MSP_ERR_UNSUPPORTED, "AMGS needs both inner and interface cells");
    std::vector<int32_t> pos(nb);
    for (int64_t i = 0; i < nb; ++i) pos[perm[i]] = static_cast<int32_t>(i);
    Csr A;
    A.nr = A.nc = nb;
    A.rp.assign(nb + 1, 0);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = 0; i < nb; ++i) {
        const int64_t g = perm[i];
        row.clear();
        for (int64_t k = sym.Ainn.rp[g]; k < sym.Ainn.rp[g + 1]; ++k) row.emplace_back(pos[sym.Ainn.ci[k]], sym.Ainn.v[k]);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) { return x.first < y.first; });
        for (auto& e : row) {
            A.ci.push_back(e.first);
            A.v.push_back(e.second);
        }
        A.rp[i + 1] = static_cast<int64_t>(A.ci.size());
    }
    std::vector<double> sigma(sym.sigma.size());
    std::vector<int64_t> img(sym.img.size());
    std::vector<int8_t> iface(nb);
    for (int64_t i = 0; i < nb; ++i) {
        for (int a = 0; a < S; ++a) {
            sigma[i * S + a] = sym.sigma[perm[i] * S + a];
            img[i * S + a] = sym.img[perm[i] * S + a];
        }
        iface[i] = i >= nI ? 1 : 0;
    }
    sym.Ainn = std::move(A);
    sym.sigma = std::move(sigma);
    sym.img = std::move(img);
    sym.iface = std::move(iface);

    AmgsParts P;
    P.nI = nI;
    P.K = block_of(sym.Ainn, 0, nI, 0, nI);
    P.B = block_of(sym.Ainn, 0, nI, nI, nb);
    P.C1 = block_of(sym.Ainn, nI, nb, nI, nb);
    P.BT = transpose(P.B);
    const double tau = o.schur_tau;
    P.GK = fsai_filtered_power(P.K, tau, 2);
    P.GKT = transpose(P.GK);
    const Csr W1 = spgemm(P.GK, P.B);
    const Csr W2 = spgemm(P.GKT, W1);
    const Csr X = spgemm(P.BT, W2);
    Csr Xs = add_csr(X, 1.0, transpose(X), 1.0);   // (X + X^T) / 2: exactly symmetric
    for (double& v : Xs.v) v *= 0.5;
    P.SG1 = add_csr(P.C1, 1.0, Xs, -1.0);
    P.GS1 = fsai_filtered_power(P.SG1, tau, 3);
    P.GS1T = transpose(P.GS1);
    P.HK = build_hierarchy(P.K, std::vector<int8_t>(nI, 0), o);
    return P;
}

SubValues replicated_sub_values(const HostHierarchy& H, int S) {
    SubValues V;
    V.S = S;
    const int L = static_cast<int>(H.lev.size());
    if (L < 2) return V;
    auto rep = [S](const std::vector<double>& v) {
        std::vector<double> out(v.size() * S);
        for (size_t k = 0; k < v.size(); ++k)
            for (int a = 0; a < S; ++a) out[k * S + a] = v[k];
        return out;
    };
    V.A.assign(L, {});
    V.P.assign(L, {});
    V.R.assign(L, {});
    V.M.assign(L, {});
    V.G.assign(L, {});
    V.omega.assign(L, std::vector<double>(S, 0.0));
    for (int l = 1; l < L; ++l) {
        V.A[l] = rep(H.lev[l].A.v);
        if (l + 1 < L) {
            V.P[l] = rep(H.lev[l].P.v);
            V.R[l] = rep(H.lev[l].R.v);
            V.M[l] = rep(H.lev[l].M.v);
            V.G[l] = rep(H.lev[l].G.v);
            V.omega[l].assign(S, H.lev[l].omega);
        }
    }
    const size_t nn = H.coarse_inv.size();
    V.coarse_inv.resize(nn * S);
    for (int a = 0; a < S; ++a) std::copy(H.coarse_inv.begin(), H.coarse_inv.end(), V.coarse_inv.begin() + a * nn);
    return V;
}

SubValues build_sub_values(const HostHierarchy& H, const std::vector<double>& sigma, const std::vector<int8_t>& iface,
                           int S, const msp_opts& o) {
    SubValues V;
    V.S = S;
    const int L = static_cast<int>(H.lev.size());
    if (L < 2) return V;
    V.A.assign(L, {});
    V.P.assign(L, {});
    V.R.assign(L, {});
    V.M.assign(L, {});
    V.G.assign(L, {});
    V.omega.assign(L, std::vector<double>(S, 0.0));
    for (int l = 1; l < L; ++l) {
        V.A[l].assign(H.lev[l].A.nnz() * S, 0.0);
        if (l + 1 < L) {
            V.P[l].assign(H.lev[l].P.nnz() * S, 0.0);
            V.R[l].assign(H.lev[l].R.nnz() * S, 0.0);
            V.M[l].assign(H.lev[l].M.nnz() * S, 0.0);
            V.G[l].assign(H.lev[l].G.nnz() * S, 0.0);
        }
    }
    const int64_t nL = H.lev[L - 1].A.nr;
    V.coarse_inv.assign(static_cast<size_t>(S) * nL * nL, 0.0);
    // coarse numbers of the reduction level
    const HostLevel& L0 = H.lev[0];
    std::vector<int32_t> cnum(L0.A.nr, -1);
    int32_t nc = 0;
    for (int64_t i = 0; i < L0.A.nr; ++i)
        if (L0.cf[i]) cnum[i] = nc++;
    std::vector<std::string> errs(S);
    auto one = [&](int a) {
        Csr A = H.lev[1].A;
        for (int64_t i = 0; i < L0.A.nr; ++i) {
            if (!iface[i]) continue;
            const int32_t j = cnum[i];
            if (j < 0) throw Error(MSP_ERR_ARG, "interface point is not coarse");
            const int32_t* b = A.ci.data() + A.rp[j];
            const int32_t* e = A.ci.data() + A.rp[j + 1];
            const int32_t* f = std::lower_bound(b, e, j);
            if (f == e || *f != j) throw Error(MSP_ERR_ARG, "missing diagonal in the reduced operator");
            double& d = A.v[f - A.ci.data()];
            d = d + sigma[static_cast<size_t>(i) * S + a];
        }
        for (int l = 1; l < L; ++l) {
            const HostLevel& Ls = H.lev[l];
            for (int64_t k = 0; k < A.nnz(); ++k) V.A[l][k * S + a] = A.v[k];
            if (l + 1 == L) break;
            std::vector<std::vector<int32_t>> lower(A.nr);
            for (int64_t i = 0; i < A.nr; ++i)
                for (int64_t k = Ls.G.rp[i]; k < Ls.G.rp[i + 1]; ++k)
                    if (Ls.G.ci[k] != i) lower[i].push_back(Ls.G.ci[k]);
            Csr G = fsai_rows(A, lower);
            Csr GT = transpose(G);
            const double om = damping(A, G, GT, o.seed);
            Csr P = interpolation(A, Ls.cf, o.jacobi);
            if (o.emin_steps > 0) emin(A, Ls.cf, P, o.emin_steps);
            Csr R = transpose(P);
            Csr M = spgemm(GT, G);
            for (double& v : M.v) v *= om;
            if (!same_pattern(P, Ls.P) || !same_pattern(M, Ls.M) || !same_pattern(G, Ls.G))
                throw Error(MSP_ERR_ARG, "subsystem level pattern differs from the shared level");
            V.omega[l][a] = om;
            for (int64_t k = 0; k < P.nnz(); ++k) V.P[l][k * S + a] = P.v[k];
            for (int64_t k = 0; k < R.nnz(); ++k) V.R[l][k * S + a] = R.v[k];
            for (int64_t k = 0; k < M.nnz(); ++k) V.M[l][k * S + a] = M.v[k];
            for (int64_t k = 0; k < G.nnz(); ++k) V.G[l][k * S + a] = G.v[k];
            Csr Anext = spgemm(R, spgemm(A, P));
            if (!same_pattern(Anext, H.lev[l + 1].A))
                throw Error(MSP_ERR_ARG, "subsystem reduced operator pattern differs from the shared one");
            A = std::move(Anext);
        }
        const std::vector<double> inv = dense_inverse(A);
        std::copy(inv.begin(), inv.end(), V.coarse_inv.begin() + static_cast<size_t>(a) * nL * nL);
    };
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> th;
    std::vector<int> codes(S, MSP_OK);
    const int share = std::max(1, setup_threads() / S);   // row loops inside a subsystem's worker
    for (int a = 0; a < S; ++a)
        th.emplace_back([&, a]() {
            t_share = share;
            try {
                one(a);
            } catch (const Error& e) {
                codes[a] = e.status;
                errs[a] = e.what();
            }
        });
    for (auto& t : th) t.join();
    for (int a = 0; a < S; ++a)
        if (codes[a] != MSP_OK) throw Error(codes[a], "subsystem " + std::to_string(a) + ": " + errs[a]);
    const char* logv = std::getenv("MSP_SETUP_LOG");
    if (logv && *logv && std::strcmp(logv, "0") != 0)
        std::fprintf(stderr, "msp setup: per-subsystem values of levels >= 1 %.3f s\n",
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    return V;
}

}  // namespace msp
