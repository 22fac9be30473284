// Host-only exercise of the library's setup code (block extraction and
// validation, the multigrid-reduction hierarchy, the per-subsystem values,
// damping and stand-alone FSAI), built with address and undefined-behaviour
// sanitizers by tests/test_host_sanitizers.py.  The problem is a cell-centred
// 7-point Poisson matrix on an nx x ny x nz grid with Dirichlet walls, a
// coefficient field that is mirror symmetric about every mid-plane, and s
// mirror symmetries (about the x, y, z mid-planes in that order).  Exit code
// 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace {

struct Grid {
    int nx, ny, nz, s;
};

int64_t cell(const Grid& g, int x, int y, int z) { return (int64_t(z) * g.ny + y) * g.nx + x; }

// coefficient of a cell: smooth and mirror symmetric about each mid-plane
double kappa(const Grid& g, int x, int y, int z) {
    const double u = std::fabs(x + 0.5 - g.nx / 2.0), v = std::fabs(y + 0.5 - g.ny / 2.0),
                 w = std::fabs(z + 0.5 - g.nz / 2.0);
    return std::exp(0.7 * std::sin(0.9 * u) + 0.5 * std::cos(1.3 * v) + 0.3 * std::sin(0.4 * w + 0.2 * u));
}

struct Full {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
    std::vector<int64_t> img;
    int64_t n = 0, n_b = 0;
};

Full assemble(const Grid& g) {
    Full F;
    F.n = int64_t(g.nx) * g.ny * g.nz;
    F.rp.push_back(0);
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x) {
                const double k0 = kappa(g, x, y, z);
                double face[6];
                std::vector<std::pair<int32_t, double>> row;
                const int d[6][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
                for (int f = 0; f < 6; ++f) {
                    const int X = x + d[f][0], Y = y + d[f][1], Z = z + d[f][2];
                    if (X < 0 || Y < 0 || Z < 0 || X >= g.nx || Y >= g.ny || Z >= g.nz) {
                        face[f] = 2.0 * k0;   // Dirichlet wall
                        continue;
                    }
                    const double k1 = kappa(g, X, Y, Z);
                    face[f] = 2.0 * k0 * k1 / (k0 + k1);
                    row.emplace_back(static_cast<int32_t>(cell(g, X, Y, Z)), -face[f]);
                }
                // opposite faces summed first: the same bits in every mirror image
                const double diag = ((face[2] + face[3]) + (face[1] + face[4])) + (face[0] + face[5]);
                row.emplace_back(static_cast<int32_t>(cell(g, x, y, z)), diag);
                for (const auto& e : row) {
                    F.ci.push_back(e.first);
                    F.v.push_back(e.second);
                }
                F.rp.push_back(static_cast<int64_t>(F.ci.size()));
            }
    // base cells: the low half along each mirrored axis; image a reflects axis t where bit t is set
    const int bx = g.s >= 1 ? g.nx / 2 : g.nx, by = g.s >= 2 ? g.ny / 2 : g.ny, bz = g.s >= 3 ? g.nz / 2 : g.nz;
    const int S = 1 << g.s;
    F.n_b = int64_t(bx) * by * bz;
    F.img.resize(static_cast<size_t>(F.n_b) * S);
    int64_t i = 0;
    for (int z = 0; z < bz; ++z)
        for (int y = 0; y < by; ++y)
            for (int x = 0; x < bx; ++x, ++i)
                for (int a = 0; a < S; ++a) {
                    const int X = (a & 1) ? g.nx - 1 - x : x, Y = (a & 2) ? g.ny - 1 - y : y,
                              Z = (a & 4) ? g.nz - 1 - z : z;
                    F.img[static_cast<size_t>(i) * S + a] = cell(g, X, Y, Z);
                }
    return F;
}

int failures = 0;

void check(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

bool csr_ok(const msp::Csr& M) {
    if (static_cast<int64_t>(M.rp.size()) != M.nr + 1 || M.rp[0] != 0) return false;
    for (int64_t r = 0; r < M.nr; ++r) {
        if (M.rp[r + 1] < M.rp[r]) return false;
        for (int64_t k = M.rp[r]; k < M.rp[r + 1]; ++k) {
            if (M.ci[k] < 0 || M.ci[k] >= M.nc) return false;
            if (k > M.rp[r] && M.ci[k] <= M.ci[k - 1]) return false;
            if (!std::isfinite(M.v[k])) return false;
        }
    }
    return M.ci.size() == static_cast<size_t>(M.nnz()) && M.v.size() == static_cast<size_t>(M.nnz());
}

void run(const Grid& g, int pc) {
    Full F = assemble(g);
    const msp_csr A{F.n, F.rp.data(), F.ci.data(), F.v.data()};
    const msp_symmap map{g.s, F.n_b, F.img.data()};
    msp_opts o;
    msp_default_opts(&o);
    o.coarse_max = 48;
    o.device = -1;
    o.pc = pc;
    const msp::SymParts P = msp::extract_blocks(&A, &map);
    check(P.n_b == F.n_b && csr_ok(P.Ainn), "inner block");
    const int S = 1 << g.s;
    const msp::HostHierarchy H = msp::build_hierarchy(P.Ainn, P.iface, o);
    check(H.lev.size() >= 2, "hierarchy depth");
    for (size_t l = 0; l < H.lev.size(); ++l) {
        const msp::HostLevel& L = H.lev[l];
        check(csr_ok(L.A), "level operator");
        if (l + 1 < H.lev.size()) {
            check(csr_ok(L.P) && csr_ok(L.R) && csr_ok(L.G) && csr_ok(L.M), "level transfer and smoother");
            check(L.P.nr == L.A.nr && L.P.nc == H.lev[l + 1].A.nr, "prolongation shape");
            check(L.omega > 0.0 && std::isfinite(L.omega), "damping");
        }
    }
    const int64_t nL = H.lev.back().A.nr;
    check(static_cast<int64_t>(H.coarse_inv.size()) == nL * nL, "coarsest inverse size");
    if (pc == MSP_PC_AMGR_SUB && H.lev.size() > 1) {
        const msp::SubValues V = msp::build_sub_values(H, P.sigma, P.iface, S, o);
        check(V.S == S && static_cast<int64_t>(V.coarse_inv.size()) == S * nL * nL, "per-subsystem coarsest");
        for (size_t l = 1; l + 1 < H.lev.size(); ++l)
            check(static_cast<int64_t>(V.P[l].size()) == H.lev[l].P.nnz() * S, "per-subsystem interpolation");
    }
    const msp::Csr G = msp::fsai_full_lower(P.Ainn);
    check(csr_ok(G), "stand-alone FSAI");
}

// Invalid inputs must come back as msp::Error with the documented status.
void rejects() {
    const Grid g{8, 6, 4, 2};
    Full F = assemble(g);
    const msp_csr A{F.n, F.rp.data(), F.ci.data(), F.v.data()};
    std::vector<int64_t> bad = F.img;
    bad[0] = bad[4];   // not a permutation
    const msp_symmap m1{g.s, F.n_b, bad.data()};
    int st = 0;
    try {
        msp::extract_blocks(&A, &m1);
    } catch (const msp::Error& e) {
        st = e.status;
    }
    check(st == MSP_ERR_BAD_MAP, "non-permutation map rejected");
    std::vector<double> v = F.v;
    v[3] += 1e-3;   // breaks exact symmetry
    const msp_csr A2{F.n, F.rp.data(), F.ci.data(), v.data()};
    const msp_symmap m2{g.s, F.n_b, F.img.data()};
    st = 0;
    try {
        msp::extract_blocks(&A2, &m2);
    } catch (const msp::Error& e) {
        st = e.status;
    }
    check(st == MSP_ERR_NOT_SYMMETRIC, "asymmetric matrix rejected");
}

}  // namespace

// FNV-1a over the bytes of every level's arrays and the per-subsystem values of a
// larger setup with the adaptive FSAI and energy minimisation: equal across thread
// counts when every row is computed with the serial arithmetic.
uint64_t fnv(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

template <typename T>
uint64_t fnv(uint64_t h, const std::vector<T>& v) {
    return fnv(h, v.data(), v.size() * sizeof(T));
}

int checksum() {
    const Grid g{48, 40, 32, 1};
    Full F = assemble(g);
    const msp_csr A{F.n, F.rp.data(), F.ci.data(), F.v.data()};
    const msp_symmap map{g.s, F.n_b, F.img.data()};
    msp_opts o;
    msp_default_opts(&o);
    o.coarse_max = 200;
    o.device = -1;
    o.pc = MSP_PC_AMGR_SUB;
    o.afsai_nnz = 5;
    o.emin_steps = 4;
    const msp::SymParts P = msp::extract_blocks(&A, &map);
    const msp::HostHierarchy H = msp::build_hierarchy(P.Ainn, P.iface, o);
    const msp::SubValues V = msp::build_sub_values(H, P.sigma, P.iface, 1 << g.s, o);
    uint64_t h = 1469598103934665603ull;
    for (const msp::HostLevel& L : H.lev) {
        for (const msp::Csr* M : {&L.A, &L.P, &L.R, &L.G, &L.GT, &L.M}) {
            h = fnv(h, M->rp);
            h = fnv(h, M->ci);
            h = fnv(h, M->v);
        }
        h = fnv(h, L.cf);
        h = fnv(h, &L.omega, sizeof(L.omega));
    }
    h = fnv(h, H.coarse_inv);
    for (const auto* X : {&V.A, &V.P, &V.R, &V.M, &V.G, &V.omega})
        for (const auto& v : *X) h = fnv(h, v);
    h = fnv(h, V.coarse_inv);
    std::printf("levels %zu checksum %016llx\n", H.lev.size(), static_cast<unsigned long long>(h));
    return 0;
}

int main(int argc, char** argv) {
    if (argc > 1 && std::strcmp(argv[1], "--checksum") == 0) return checksum();
    run(Grid{16, 12, 10, 3}, MSP_PC_AMGR_SUB);
    run(Grid{20, 14, 8, 2}, MSP_PC_AMGR);
    run(Grid{24, 16, 1, 1}, MSP_PC_AMGR_SUB);
    rejects();
    if (failures) return 1;
    std::printf("host setup checks passed\n");
    return 0;
}
