// Internal data structures of the mirror-symmetric Poisson library.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "msp.h"

namespace msp {

// Error carried to the C boundary as (status, message).
struct Error : std::runtime_error {
    int status;
    Error(int st, const std::string& msg) : std::runtime_error(msg), status(st) {}
};

// Host CSR, sorted columns, 64-bit row pointers.
struct Csr {
    int64_t nr = 0, nc = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
    int64_t nnz() const { return rp.empty() ? 0 : rp[nr]; }
};

Csr transpose(const Csr& A);
// Entry p of transpose(A) is entry map[p] of A.
std::vector<int64_t> transpose_map(const Csr& A);
// Symbolic patterns of the interpolation's Jacobi steps W_1 .. W_steps (rows:
// the F points in increasing order; columns: coarse numbers), as the
// interpolation builds them before any truncation; values left empty.
std::vector<Csr> interpolation_patterns(const Csr& A, const std::vector<int8_t>& cf, int steps);
// Product with the structural pattern (explicit zeros kept); each value is
// sum_k A_ik B_kj accumulated in increasing k (Gustavson order).
Csr spgemm(const Csr& A, const Csr& B);

// One level of the shared hierarchy (host copy).
struct HostLevel {
    Csr A;
    std::vector<int8_t> cf;   // 1 = coarse (empty on the coarsest level)
    Csr P, R, G, GT;
    Csr M;                    // smoother omega * G^T G, formed explicitly
    double omega = 0.0;
};

struct HostHierarchy {
    std::vector<HostLevel> lev;
    std::vector<double> coarse_inv;   // dense inverse of the coarsest A, row-major
};

// Per-subsystem values of the levels below the reduction (AMGR on every
// decoupled subsystem): level l >= 1 of subsystem a has the patterns of the
// shared level l (same C/F split and smoother pattern) and its own values.
// Values are interleaved, entry k of subsystem a at [k * S + a].
struct SubValues {
    int S = 0;
    std::vector<std::vector<double>> A, P, R, M, G;   // by level (index 0 unused)
    std::vector<std::vector<double>> omega;           // by level, S values
    std::vector<double> coarse_inv;                   // S blocks of nL x nL
};

// A_1,a = A_1,inn + diag(sigma_a on the interface coarse points), then the
// standard levels with the shared splits and patterns.
SubValues build_sub_values(const HostHierarchy& H, const std::vector<double>& sigma,
                           const std::vector<int8_t>& iface, int S, const msp_opts& o);
// Every subsystem holding the shared levels' values (the layout of build_sub_values):
// storage for values that a device re-setup computes afterwards.
SubValues replicated_sub_values(const HostHierarchy& H, int S);

// Result of block extraction (Sec. 2).
struct SymParts {
    int s = 0;
    int64_t n = 0, n_b = 0;
    Csr Ainn;                       // H_0
    std::vector<double> sigma;      // n_b * 2^s, diagonal of A_out,a
    std::vector<int8_t> iface;      // n_b
    std::vector<int64_t> img;       // n_b * 2^s
    // where the values come from in the caller's CSR arrays (the numeric re-setup
    // gathers a new matrix's values through these): A_inn entry k <- inn_src[k];
    // outer coupling j of base cell i <- out_src[i * (2^s - 1) + j - 1] (-1: none)
    std::vector<int64_t> inn_src, out_src;
    int64_t src_nnz = 0;
};

SymParts extract_blocks(const msp_csr* A, const msp_symmap* map);

// A domain made of copies of one subdomain, solved in its own ordering: the
// parts of a one-subsystem context (s = 0, identity map, no outer diagonal)
// plus the interface of the copies and the replicated level-0 split.
struct CopyParts {
    SymParts sym;                  // Ainn = the whole matrix; iface over all n unknowns
    Csr A00;                       // the base copy's block, base numbering
    std::vector<int8_t> iface_base;
    std::vector<int8_t> cf0;       // populated interface over all n unknowns
};
CopyParts extract_copies(const msp_csr* A, const msp_copies* map, const msp_opts& o);

// Alg. 2 on A with the given interface (MIS of T^d over the inner nodes, joined
// with the interface); 1 = coarse.
std::vector<int8_t> reduction_split(const Csr& A, const std::vector<int8_t>& iface, const msp_opts& o);
// cf0: a level-0 split computed elsewhere, used instead of Alg. 2 on Ainn.
HostHierarchy build_hierarchy(const Csr& Ainn, const std::vector<int8_t>& iface, const msp_opts& o,
                              const std::vector<int8_t>* cf0 = nullptr);
// The reduction level of `old` as it is (split, patterns and values), every level
// below it built afresh from old's level-1 operator, as build_hierarchy builds them.
HostHierarchy build_hierarchy_below(const HostHierarchy& old, const msp_opts& o);
// AMGS, the Schur-complement AMG of Sec. 3.1, on the decoupled subsystems:
// base cells reordered inner first (eq. (3.1)), so K = A_inn[0:nI, 0:nI],
// B = A_inn[0:nI, nI:], C_1 = A_inn[nI:, nI:]; the AMG of K (HK); the FSAI of K
// (GK, eq. (3.4)); S_G1 = C_1 - sym(B^T G_K^T G_K B) and its FSAI (GS1,
// eq. (3.9)).  FSAI patterns: the lower triangle of the pattern of K_f^2 and
// of S_f^3, M_f = M without the off-diagonal entries |m_ij| < tau sqrt(|m_ii m_jj|).
struct AmgsParts {
    int64_t nI = 0;
    Csr K, B, BT, C1, GK, GKT, SG1, GS1, GS1T;
    HostHierarchy HK;
};
// Reorders sym's base cells inner first (stable) and builds the parts.
AmgsParts build_amgs(SymParts& sym, const msp_opts& o);

// omega = 4/(3 lam), lam from 20 power iterations on G A G^T (seeded start).
double damping(const Csr& A, const Csr& G, const Csr& GT, uint64_t seed);
// Static FSAI on the full lower pattern of A (the stand-alone FSAI of A_inn).
Csr fsai_full_lower(const Csr& A);

// finite-volume operator (fv.cpp)
void fv_create(const msp_faces* F, const msp_symmap* map, int device, msp_fv** out);
int64_t fv_nnz(const msp_fv* f);
void fv_assemble(const msp_fv* f, const double* kappa_base, int64_t* rp, int32_t* ci, double* va);
void fv_free(msp_fv* f);

uint64_t splitmix64(uint64_t x);
double unit_centered(uint64_t x);

// Dense symmetric eigen-decomposition (cyclic Jacobi), row-major n x n input;
// eigenvalues ascending, eigenvectors as columns of V (row-major).
void sym_eig(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& V);

}  // namespace msp
