// C interface, device context and the solve driver (Alg. 1 with per-column
// PCG; the shared preconditioner applied to every column at once).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <numeric>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "pcg.hpp"
#include "refresh.hpp"

namespace msp {

static thread_local std::string g_last_error;

#define HIPCHECK(expr)                                                                                 \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            throw msp::Error(e_ == hipErrorOutOfMemory ? MSP_ERR_OOM : MSP_ERR_HIP,                    \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                            \
    } while (0)

// Sliced-ELL form of a matrix for one row split G (sell.hip).
struct DevSell {
    int G = 0;               // 0 = not built
    int64_t slots = 0;
    int64_t* off = nullptr;  // first slot of each slice of 64 virtual rows
    int32_t* wid = nullptr;  // width of each slice
    int32_t* ci = nullptr;   // column per slot, -1 for padding
    double* v64 = nullptr;   // values per slot (vs interleaved sets)
    float* v32 = nullptr;
    int64_t* pos = nullptr;  // CSR entry per slot, -1 for padding (built by the first re-setup)
};
constexpr int kSellForms = 5;   // G = 1, 2, 4, 8, 16

// Device CSR: 32-bit row pointers and columns, FP64 and (mixed modes) FP32 values.
struct DevCsr {
    int64_t nr = 0, nc = 0, nnz = 0;
    int split = 1;           // lane groups per row (long rows are split)
    int vs = 1;              // interleaved value sets (one per subsystem), entry k of set a at k * vs + a
    int tuned[3][7] = {};    // autotuned split by [multivector type: FP64, FP32, BF16][log2 C]; 0 = not tuned
    bool wide[3][7] = {};    // autotuned 16-byte lanes of the one-group kernel, same indexing
    int sg[3][7] = {};       // autotuned: 0 = CSR kernels, else the row split G of the sliced-ELL kernel
    const Csr* hpat = nullptr;                  // host pattern and values (V-cycle matrices: the sliced
    const std::vector<double>* hval = nullptr;  // forms are built from them when the autotuner needs them)
    bool f32 = false;                           // FP32 values on the device (mixed modes)
    DevSell sell[kSellForms];
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    double* v64 = nullptr;
    float* v32 = nullptr;
    Bf16* v16 = nullptr;      // bfloat16 values (smoother in the BF16 variant)
};

// Outer diagonal on the device (OuterDiag) with its size for the byte counts.
struct DevOuter {
    OuterDiag d{nullptr, nullptr};
    int64_t rows = 0;     // rows of the operator
    int64_t carried = 0;  // rows with an outer term
};

struct DevLevel {
    DevCsr A, P, R, M;
    DevCsr G, GT;             // bfloat16 FSAI factors (BF16 variant only)
    double omega = 0.0;
    int64_t n = 0;
};

constexpr int kMaxLevels = 32;   // hierarchy depth the workspace and the statistics hold

// Pinned host memory the solve reads flags and statistics into.
struct HostBufs {
    int* h_flags = nullptr;   // pinned host copy of flags
    int* h_pub = nullptr;     // fine-grained host memory the device publishes flags into: flags, sequence number
    int* d_pub = nullptr;     // its device-visible address
    int* h_iters = nullptr;
    double* h_scal = nullptr;
};

// Column-count-dependent workspace.  Every device array is carved from one
// block (carve_work): the library's own allocation for msp_solve_device, the
// static scratch array for the allocation-free entry point.
struct Work {
    int C = 0;
    int m = 1;                // columns per subsystem of the current solve
    double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *zold = nullptr;
    void* vy[kMaxLevels] = {};   // per level, element type of the V-cycle
    void* vs[kMaxLevels] = {};
    void* vr[kMaxLevels] = {};
    void* vt[kMaxLevels] = {};   // factored smoother (BF16-G variant)
    double* partial = nullptr;
    int nb_dot = 0;
    int grid_op = 0, grid_upd = 0, grid_z = 0, grid_p = 0;   // PCG kernel grids (set by the first solve plan)
    double *amgs1 = nullptr, *amgs2 = nullptr;   // pc = AMGS: two n_b x C scratch multivectors
    double* dense_part = nullptr;   // k-chunk partials of the dense coarsest solve
    void* dense_pack = nullptr;     // per-subsystem packed right-hand sides of the coarsest solves
    int dense_rows = 8;             // rows per wavefront of the per-subsystem coarsest solves (autotuned)
    // partials of the fused PCG kernels: two column sets and the low-rank projections
    double *pp1 = nullptr, *pp2 = nullptr, *plrc = nullptr;
    double* scal = nullptr;   // SC_COUNT arrays of 64
    int* iscal = nullptr;     // active[64], iters[64], flags[2]
    int* h_flags = nullptr;   // host buffers (HostBufs of the workspace or of the context)
    int* h_pub = nullptr;
    int* d_pub = nullptr;
    int pub_seq = 0;
    int* h_iters = nullptr;
    double* h_scal = nullptr;
    HostBufs own;             // pinned buffers this workspace allocated (freed with the context)
};

enum { SC_RR = 0, SC_RZ, SC_PQ, SC_RHO, SC_ALPHA, SC_BETA, SC_THR, SC_RNORM, SC_BN2, SC_TRUE, SC_COUNT };

// Device structure of the numeric re-setup (built by the first msp_refresh).
struct RfPat {
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    int64_t nr = 0, nnz = 0;
};
struct RfLevel {
    int64_t n = 0, nf = 0;
    RfPat A, G, GT, M, P, R, AP;     // A, M, P, R share the V-cycle matrices' patterns
    std::vector<RfPat> W;            // Jacobi steps of the interpolation (F rows)
    int32_t* fidx = nullptr;
    int8_t* cf = nullptr;
    int32_t* cnum = nullptr;
    int32_t* fnum = nullptr;
    int32_t* pmap = nullptr;         // P entry -> entry of the last Jacobi step (F rows)
    int64_t* gt_src = nullptr;       // G^T entry -> G entry
    int64_t* r_src = nullptr;        // R entry -> P entry
    int64_t* woff = nullptr;         // FSAI workspace offsets
    double* v0 = nullptr;            // normalised start vector of the damping's power iteration
    double *a = nullptr, *g = nullptr, *gt = nullptr, *m = nullptr, *p = nullptr, *r = nullptr, *ap = nullptr;
    std::vector<double*> w;
    double* afc = nullptr;
    int8_t* hasf = nullptr;
    double omega = 0.0;
};
struct SplitCheck {              // one level's split redone on the device for new values
    bool on = false;
    int d = 1;                       // independent-set distance
    RfPat A;                         // the level's operator pattern (symmetric)
    int64_t* tmap = nullptr;         // entry (i, j) -> entry (j, i)
    uint64_t* pri = nullptr;         // hash priorities
    int32_t* lam = nullptr;          // strong dependants (levels below the reduction; nullptr at level 0)
    int8_t *smask = nullptr, *tmask = nullptr, *state = nullptr, *state_init = nullptr, *cf = nullptr;
};
struct RefreshState {
    int64_t* inn_src = nullptr;
    int64_t* out_src = nullptr;
    double* sigma = nullptr;                  // n_b x S
    int64_t* dsig_src = nullptr;              // compact outer-diagonal values <- sigma entries
    int64_t ndsig = 0;
    int64_t* dsig1_src = nullptr;
    int64_t ndsig1 = 0;
    int64_t* s1_diag = nullptr;               // A_1 diagonal entries of the interface's coarse points
    int64_t* s1_base = nullptr;               // and their base cells
    int64_t ns1 = 0;
    std::vector<RfLevel> lev;
    double* work = nullptr;
    double *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;
    double* part = nullptr;
    double* dots = nullptr;
    int nbp = 256;
    double *dense = nullptr, *rowk = nullptr, *colk = nullptr;
    double* sets = nullptr;                   // coarsest operators of every subsystem, interleaved
    double* shared1 = nullptr;                // per-subsystem mode: shared A_1 (without the outer diagonal)
    double* sub_a1 = nullptr;                 // and A_1,a, the FSAI factors of every subsystem, interleaved
    std::vector<double*> sub_g;
    bool shared_stale = false;                // shared levels below the reduction level not recomputed yet
    // the splits of levels 0 and 1 for the new values, compared with the kept ones
    SplitCheck sc0, sc1;
    int* left = nullptr;
    unsigned long long* diff = nullptr;
    int emin_steps = 0;                       // energy minimisation of the interpolations (as the setup)
    double* em[6] = {};                       // its work vectors over P's entries
    double* gf = nullptr;                     // pc = FSAI: FSAI of A_inn and its transpose map
    int64_t* gft_src = nullptr;
    int64_t* gf_woff = nullptr;
    RfPat gfp, gftp;
    int* err = nullptr;
};

// Launch classes for the optional per-kernel timers (msp_set_timing).
enum {
    KD_OP = 0,        // q = (A_inn + outer diagonal) p
    KD_DOT = 1,       // per-column dot products (partials + reduction)
    KD_UPDATE = 2,    // r -= alpha q with <r,r>, <r,z_old>, U^T r
    KD_PUPDATE = 3,   // x += alpha p, p = z + beta p
    KD_QS = 4,        // Q_s butterflies
    KD_CAST = 5,      // precision casts at the preconditioner boundary
    KD_DENSE = 6,     // coarsest-level dense solve
    KD_FSAI = 7,      // FSAI preconditioner products
    KD_LRC = 8,       // low-rank corrections
    KD_AMGS = 9,      // AMGS: products with B, B^T and the FSAI factors of K and S_G1
    KD_LEVEL = 16,    // + 8 * level + {0: A, 1: G, 2: G^T, 3: R, 4: P}
    KD_COUNT = 16 + 8 * 20
};

struct PendingTime {
    int kind;
    double bytes;
    hipEvent_t e0, e1;
};

struct Timers {
    std::vector<char> on = std::vector<char>(KD_COUNT, 0);
    std::vector<int64_t> count = std::vector<int64_t>(KD_COUNT, 0);
    std::vector<double> ms = std::vector<double>(KD_COUNT, 0.0);
    std::vector<double> bytes = std::vector<double>(KD_COUNT, 0.0);
    std::vector<std::string> variant = std::vector<std::string>(KD_COUNT);   // kernel(s) of the last timed launch
    std::vector<PendingTime> pending;
    std::vector<hipEvent_t> pool;
};

}  // namespace msp

struct msp_ctx {
    msp_opts o{};
    msp::SymParts sym;
    msp::HostHierarchy hier;
    msp::SubValues subv;      // per-subsystem values of levels >= 1 (pc = AMGR_SUB)
    bool sub = false;         // levels >= 1 and the coarsest solve are per subsystem
    msp::Csr Gf;              // FSAI of A_inn (pc = FSAI)
    msp::AmgsParts am;        // pc = AMGS: blocks, FSAI factors (the AMG of K is `hier`)
    msp::DevCsr dB, dBT, dC1, dGK, dGKT, dGS1, dGS1T;
    msp::DevOuter dsigG;      // pc = AMGS: the outer diagonal on the interface rows
    double* d_ones = nullptr; // 64 ones (column coefficients of a plain subtraction)
    msp_stats stats{};
    bool on_device = false;
    int device = -1;
    std::vector<void*> allocs;
    int64_t* d_img = nullptr;
    msp::DevOuter dsig;       // outer diagonal of the base rows (compact: interface rows only)
    msp::DevOuter dsig1;      // pc = AMGR_SUB: the same at level 1 (the interface's coarse numbers)
    msp::DevCsr dAinn, dGf, dGfT;
    int op_sell[7] = {-1, -1, -1, -1, -1, -1, -1};   // operator kernel by log2 C: -1 not tuned, 0 CSR, 1 sliced
    const int* gate = nullptr;   // while a batch captures this system's iterations: its active flags (kernel gate)
    std::vector<msp::DevLevel> dl;
    double* d_cinv = nullptr;
    float* d_cinv32 = nullptr;    // per-subsystem coarsest inverses in FP32 (mixed modes), rows padded to 4
    int64_t nL = 0;
    std::map<int, std::unique_ptr<msp::Work>> works;   // by padded column count
    msp::HostBufs nohb;       // pinned host buffers of the allocation-free solves (allocated at setup)
    int nopub_seq = 0;
    // low-rank corrections: U (n_b x S*k, FP64 or FP32), coefficients (S*k)
    int lrc_k = 0;
    void* d_U = nullptr;
    bool U32 = false;             // U in FP32 (mixed modes)
    bool U16 = false;             // U in bfloat16 (bfloat16-multivector mode with AMGR)
    double* d_lrc_coef = nullptr;
    double* d_lrc_part = nullptr;
    double* d_lrc_W = nullptr;
    int lrc_nb = 0;
    std::vector<int32_t> lrc_kept;
    std::vector<double> lrc_ritz;
    msp::Timers tm;
    std::unique_ptr<msp::RefreshState> rf;   // numeric re-setup structure (first msp_refresh)
    bool host_stale = false;                 // host copy of the values older than the device's (msp::sync_host)
    bool values_invalid = false;             // a re-setup failed part way: no solve until one succeeds
    bool copies = false;                     // a domain of copies (level-0 split replicated, not Alg. 2 on A_inn)

    ~msp_ctx() {
        if (on_device) {
            (void)hipSetDevice(device);
            for (auto& p : tm.pending) {
                (void)hipEventDestroy(p.e0);
                (void)hipEventDestroy(p.e1);
            }
            for (auto e : tm.pool) (void)hipEventDestroy(e);
            for (void* p : allocs) (void)hipFree(p);
            auto free_host = [](msp::HostBufs& h) {
                if (h.h_flags) (void)hipHostFree(h.h_flags);
                if (h.h_pub) (void)hipHostFree(h.h_pub);
                if (h.h_iters) (void)hipHostFree(h.h_iters);
                if (h.h_scal) (void)hipHostFree(h.h_scal);
            };
            for (auto& kv : works) free_host(kv.second->own);
            free_host(nohb);
        }
    }

    template <typename T>
    T* dalloc(int64_t count) {
        if (count <= 0) count = 1;
        void* p = nullptr;
        HIPCHECK(hipMalloc(&p, sizeof(T) * static_cast<size_t>(count)));
        allocs.push_back(p);
        return static_cast<T*>(p);
    }
    void dfree(void* p) {
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) {
            allocs.erase(it);
            (void)hipFree(p);
        }
    }
    template <typename T>
    T* upload(const T* h, int64_t count) {
        T* d = dalloc<T>(count);
        if (count > 0) HIPCHECK(hipMemcpy(d, h, sizeof(T) * static_cast<size_t>(count), hipMemcpyHostToDevice));
        return d;
    }
};

namespace msp {

// round-to-nearest-even binary32 -> bfloat16 (finite inputs)
static Bf16 to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return Bf16{static_cast<uint16_t>(r >> 16)};
}

// value of a double after rounding to FP32 then to bfloat16
static double bf16_value(double v) {
    const Bf16 h = to_bf16(static_cast<float>(v));
    const uint32_t u = static_cast<uint32_t>(h.bits) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

static DevCsr upload_csr(msp_ctx* c, const Csr& M, bool fp32, bool bf16 = false) {
    DevCsr D;
    D.nr = M.nr;
    D.nc = M.nc;
    D.nnz = M.nnz();
    if (D.nnz >= (int64_t(1) << 31)) throw Error(MSP_ERR_UNSUPPORTED, "matrix too large for 32-bit indices");
    std::vector<int32_t> rp(M.nr + 1);
    for (int64_t i = 0; i <= M.nr; ++i) rp[i] = static_cast<int32_t>(M.rp[i]);
    D.rp = c->upload(rp.data(), M.nr + 1);
    D.ci = c->upload(M.ci.data(), D.nnz);
    D.v64 = c->upload(M.v.data(), D.nnz);
    // share long rows between lane groups: about 4 entries per group
    const double avg = M.nr > 0 ? static_cast<double>(D.nnz) / static_cast<double>(M.nr) : 0.0;
    D.split = 1;
    while (D.split < 64 && 4.0 * D.split * 2 <= avg) D.split *= 2;
    if (fp32) {
        std::vector<float> f(M.v.begin(), M.v.end());
        D.v32 = c->upload(f.data(), D.nnz);
        if (bf16) {
            std::vector<Bf16> h(f.size());
            for (size_t q = 0; q < f.size(); ++q) h[q] = to_bf16(f[q]);
            D.v16 = c->upload(h.data(), D.nnz);
        }
    }
    return D;
}

// Pattern of M with vs interleaved value sets (values: nnz * vs, entry k of set a at k * vs + a).
static DevCsr upload_sets(msp_ctx* c, const Csr& M, const std::vector<double>& values, int vs, bool fp32) {
    if (static_cast<int64_t>(values.size()) != M.nnz() * vs) throw Error(MSP_ERR_ARG, "value sets size mismatch");
    Csr pat = M;
    pat.v.assign(1, 0.0);
    DevCsr D;
    D.nr = M.nr;
    D.nc = M.nc;
    D.nnz = M.nnz();
    D.vs = vs;
    if (D.nnz >= (int64_t(1) << 31) / vs) throw Error(MSP_ERR_UNSUPPORTED, "matrix too large for 32-bit indices");
    std::vector<int32_t> rp(M.nr + 1);
    for (int64_t i = 0; i <= M.nr; ++i) rp[i] = static_cast<int32_t>(M.rp[i]);
    D.rp = c->upload(rp.data(), M.nr + 1);
    D.ci = c->upload(M.ci.data(), D.nnz);
    D.v64 = c->upload(values.data(), static_cast<int64_t>(values.size()));
    const double avg = M.nr > 0 ? static_cast<double>(D.nnz) / static_cast<double>(M.nr) : 0.0;
    D.split = 1;
    while (D.split < 64 && 4.0 * D.split * 2 <= avg) D.split *= 2;
    if (fp32) {
        std::vector<float> f(values.begin(), values.end());
        D.v32 = c->upload(f.data(), static_cast<int64_t>(f.size()));
    }
    return D;
}

// matrix values used with multivectors of type T (bfloat16 multivectors take FP32 values)
template <typename T>
struct ValOf {
    using type = T;
};
template <>
struct ValOf<Bf16> {
    using type = float;
};
template <typename T>
static const typename ValOf<T>::type* vals(const DevCsr& M);
template <>
const double* vals<double>(const DevCsr& M) { return M.v64; }
template <>
const float* vals<float>(const DevCsr& M) { return M.v32; }
template <>
const float* vals<Bf16>(const DevCsr& M) { return M.v32; }

template <typename T>
static int tslot() {
    return sizeof(T) == 8 ? 0 : (sizeof(T) == 4 ? 1 : 2);
}

// short type names for the kernel names the timers report
template <typename T>
static const char* tname() {
    return std::is_same<T, double>::value ? "double" : (std::is_same<T, float>::value ? "float" : "Bf16");
}

static hipEvent_t take_event(msp_ctx* c) {
    if (!c->tm.pool.empty()) {
        hipEvent_t e = c->tm.pool.back();
        c->tm.pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    return e;
}

// Run `launch` bracketed by events on `st` when timers for `kind` are on;
// name() gives the kernel function(s) the launch runs (evaluated only then).
template <typename F, typename N>
static void timed(msp_ctx* c, int kind, double bytes, hipStream_t st, F&& launch, N&& name) {
    if (kind < 0 || kind >= KD_COUNT || !c->tm.on[kind]) {
        launch();
        return;
    }
    c->tm.variant[kind] = name();
    PendingTime p{kind, bytes, take_event(c), take_event(c)};
    HIPCHECK(hipEventRecord(p.e0, st));
    launch();
    HIPCHECK(hipEventRecord(p.e1, st));
    c->tm.pending.push_back(p);
}

// Fold finished event pairs into the per-kind totals (after a stream sync).
static void resolve_timers(msp_ctx* c) {
    for (auto& p : c->tm.pending) {
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, p.e0, p.e1));
        c->tm.count[p.kind] += 1;
        c->tm.ms[p.kind] += ms;
        c->tm.bytes[p.kind] += p.bytes;
        c->tm.pool.push_back(p.e0);
        c->tm.pool.push_back(p.e1);
    }
    c->tm.pending.clear();
}

// V-cycle kinds: the level products and the dense coarsest solve
static bool is_vcycle_kind(int kind) { return kind >= KD_LEVEL || kind == KD_DENSE; }
static bool vcycle_timed(const msp_ctx* c) {
    for (int k = 0; k < KD_COUNT; ++k)
        if (is_vcycle_kind(k) && c->tm.on[k]) return true;
    return false;
}
static double vcycle_ms(const msp_ctx* c) {
    double t = 0.0;
    for (int k = 0; k < KD_COUNT; ++k)
        if (is_vcycle_kind(k)) t += c->tm.ms[k];
    return t;
}

// Algorithmic bytes of Y = alpha (M X) + beta Z: the matrix once, X once,
// Y written once, Z read once if present, the outer diagonal once.
template <typename T>
static double spmm_bytes(const DevCsr& M, int C, bool z, const DevOuter* sig, int S) {
    const double w = sizeof(T);
    const double wv = (sizeof(T) == 4 && M.v16) ? 2.0 : static_cast<double>(sizeof(typename ValOf<T>::type));
    double b = static_cast<double>(M.nnz) * (wv * M.vs + 4.0) + 4.0 * static_cast<double>(M.nr + 1);
    b += static_cast<double>(M.nc) * C * w + static_cast<double>(M.nr) * C * w;
    if (z) b += static_cast<double>(M.nr) * C * w;
    if (sig) b += 4.0 * static_cast<double>(sig->rows) + 8.0 * static_cast<double>(sig->carried) * S;
    return b;
}

static int log2i(int C) {
    int l = 0;
    while ((1 << l) < C) ++l;
    return l;
}

static int log2i(int C);

// One SpMM launch with an explicit lane-group split (1 = one group per row),
// or on the sliced-ELL form with row split sg > 0; FP32 products use the
// bfloat16 values when the matrix carries them.
template <typename T>
static void spmm_launch(hipStream_t st, int C, const DevCsr& M, int split, bool wide, const T* X, T* Y, const T* Z,
                        acc_t<T> alpha, acc_t<T> beta, OuterDiag sigma, int S, int m, int sg = 0,
                        const int* gate = nullptr) {
    using TV = typename ValOf<T>::type;
    if (sg > 0) {
        const DevSell& F = M.sell[log2i(sg)];
        if (F.G != sg) throw Error(MSP_ERR_ARG, "sliced form not built");
        const TV* va;
        if constexpr (std::is_same<TV, double>::value) va = F.v64;
        else va = F.v32;
        HIPCHECK((launch_sell<T, TV>(st, C, sg, M.nr, F.off, F.wid, F.ci, va, X, Y, Z, alpha, beta, sigma, S, m, M.vs,
                                     wide, gate)));
        return;
    }
    if constexpr (std::is_same<T, float>::value) {
        if (M.v16) {
            if (split > 1)
                HIPCHECK((launch_spmm_split<float, Bf16>(st, C, split, M.nr, M.rp, M.ci, M.v16, X, Y, Z, alpha, beta,
                                                         1, m, sigma, S, gate)));
            else
                HIPCHECK((launch_spmm<float, Bf16>(st, C, M.nr, M.rp, M.ci, M.v16, X, Y, Z, alpha, beta, sigma, S, m,
                                                   1, wide, gate)));
            return;
        }
    }
    if (split > 1)
        HIPCHECK((launch_spmm_split<T, TV>(st, C, split, M.nr, M.rp, M.ci, vals<T>(M), X, Y, Z, alpha, beta, M.vs, m,
                                           sigma, S, gate)));
    else
        HIPCHECK((launch_spmm<T, TV>(st, C, M.nr, M.rp, M.ci, vals<T>(M), X, Y, Z, alpha, beta, sigma, S, m, M.vs,
                                     wide, gate)));
}

template <typename T>
static void spmm(msp_ctx* c, int kind, hipStream_t st, int C, const DevCsr& M, const T* X, T* Y, const T* Z,
                 acc_t<T> alpha, acc_t<T> beta, const DevOuter* sigma = nullptr, int S = 1, int m = 1) {
    const double bytes = c->tm.on[kind] ? spmm_bytes<T>(M, C, Z != nullptr, sigma, S) : 0.0;
    const OuterDiag od = sigma ? sigma->d : OuterDiag{nullptr, nullptr};
    const int tuned = M.tuned[tslot<T>()][log2i(C)];
    const int split = tuned ? tuned : M.split;
    const bool wide = tuned && M.wide[tslot<T>()][log2i(C)];
    const int sg = tuned ? M.sg[tslot<T>()][log2i(C)] : 0;
    timed(c, kind, bytes, st,
          [&] { spmm_launch<T>(st, C, M, split, wide, X, Y, Z, alpha, beta, od, S, m, sg, c->gate); },
          [&] {
              // the instance spmm_launch picks (bfloat16 values only for FP32 products of the BF16-G variant)
              const char* tv = (std::is_same<T, float>::value && M.v16) ? "Bf16" : tname<typename ValOf<T>::type>();
              const std::string ty = std::string(tname<T>()) + ", " + tv + ", " + std::to_string(C);
              const bool sets = M.vs > 1;
              const bool w = wide && !sets && spmm_has_wide(C, static_cast<int>(sizeof(T)));
              if (sg > 0)
                  return "k_sell<" + ty + ", " + std::to_string(sg) + ", " + (sets ? "true" : "false") + ", " +
                         (w ? "true" : "false") + ">";
              if (split > 1)
                  return "k_spmm_split<" + ty + ", " + std::to_string(split) + ", " + (sets ? "true" : "false") + ">";
              return "k_spmm<" + ty + ", " + (sets ? "true" : "false") + ", " + (wide && !sets ? "true" : "false") +
                     ">";
          });
}

static bool mixed(const msp_ctx* c) { return c->o.precision != MSP_FP64; }

// Per-subsystem coarsest solves with R rows per wavefront: FP64 inverses for
// the FP64 V-cycle, FP32 ones for the mixed modes.
template <typename T>
static void dense_sets(const msp_ctx* c, const Work& w, hipStream_t st, int m, const T* y, T* s, int R) {
    const int S = 1 << c->sym.s;
    if constexpr (std::is_same<T, double>::value) {
        if (!c->d_cinv) throw Error(MSP_ERR_UNSUPPORTED, "FP64 coarsest inverses not on the device");
        HIPCHECK((launch_dense_sets<double, double>(st, w.C, S, m, c->nL, c->d_cinv, y, s,
                                                    static_cast<double*>(w.dense_pack), R, c->gate)));
    } else if (c->d_cinv32) {
        HIPCHECK((launch_dense_sets<T, float>(st, w.C, S, m, c->nL, c->d_cinv32, y, s, static_cast<T*>(w.dense_pack),
                                              R, c->gate)));
    } else {   // FP64 inverses applied to the reduced-precision vectors (sums in FP64)
        if (!c->d_cinv) throw Error(MSP_ERR_UNSUPPORTED, "coarsest inverses not on the device");
        HIPCHECK((launch_dense_sets<T, double>(st, w.C, S, m, c->nL, c->d_cinv, y, s, static_cast<T*>(w.dense_pack),
                                               R, c->gate)));
    }
}

// bytes of the per-subsystem coarsest solves (inverses and the y, s multivectors)
template <typename T>
static double dense_sets_bytes(const msp_ctx* c, int C) {
    const int S = 1 << c->sym.s;
    const double eb = (std::is_same<T, double>::value || !c->d_cinv32) ? 8.0 : 4.0;
    return eb * S * c->nL * dense_sets_ld(c->nL, (int)eb) + 2.0 * sizeof(T) * c->nL * C;
}

// Integer value of an environment variable, or -1 when unset or not a number.
static int env_int(const char* name) {
    const char* v = std::getenv(name);
    if (!v || !*v) return -1;
    char* end = nullptr;
    const long x = std::strtol(v, &end, 10);
    return (end && *end == 0 && x >= 0 && x < (1 << 20)) ? static_cast<int>(x) : -1;
}

// Slot layout of the sliced-ELL form of pattern P with rows split into G
// virtual rows (layout in sell.hip): per slice of 64 virtual rows its first
// slot and width, and per slot the CSR entry it holds (-1: padding).
static void sell_layout(const Csr& P, int G, std::vector<int64_t>& off, std::vector<int32_t>& wid,
                        std::vector<int64_t>& pos) {
    const int64_t nv = P.nr * G, ns = (nv + 63) / 64;
    off.assign(static_cast<size_t>(ns) + 1, 0);
    wid.assign(static_cast<size_t>(ns), 0);
    for (int64_t v = 0; v < nv; ++v) {
        const int64_t r = v / G, g = v % G;
        const int64_t len = P.rp[r + 1] - P.rp[r];
        const int64_t cnt = len > g ? (len - g + G - 1) / G : 0;
        wid[v / 64] = std::max(wid[v / 64], static_cast<int32_t>(cnt));
    }
    for (int64_t q = 0; q < ns; ++q) off[q + 1] = off[q] + 64 * static_cast<int64_t>(wid[q]);
    pos.assign(static_cast<size_t>(off[ns]), -1);
    for (int64_t r = 0; r < P.nr; ++r)
        for (int64_t j = 0; j < P.rp[r + 1] - P.rp[r]; ++j) {
            const int64_t v = r * G + j % G, k = j / G;
            pos[off[v / 64] + 64 * k + v % 64] = P.rp[r] + j;
        }
}

void sync_host(msp_ctx* c);   // host copy of the values after a device re-setup (below)

// Sliced-ELL form of M with rows split into G virtual rows, built from the
// host pattern and values and uploaded with the value type the context's
// V-cycle uses.
static void build_sell(msp_ctx* c, DevCsr& M, int G) {
    DevSell& F = M.sell[log2i(G)];
    if (F.G == G) return;
    if (!M.hpat || !M.hval) throw Error(MSP_ERR_ARG, "no host copy of the matrix for the sliced form");
    sync_host(c);
    const Csr& P = *M.hpat;
    const std::vector<double>& V = *M.hval;
    const int vs = M.vs;
    std::vector<int64_t> off, pos;
    std::vector<int32_t> wid;
    sell_layout(P, G, off, wid, pos);
    const int64_t ns = static_cast<int64_t>(wid.size()), slots = off[ns];
    std::vector<int32_t> ci(static_cast<size_t>(slots), -1);
    std::vector<double> val(static_cast<size_t>(slots) * vs, 0.0);
    for (int64_t q = 0; q < slots; ++q) {
        const int64_t p = pos[q];
        if (p < 0) continue;
        ci[q] = P.ci[p];
        for (int a = 0; a < vs; ++a) val[q * vs + a] = V[p * vs + a];
    }
    F.off = c->upload(off.data(), ns + 1);
    F.wid = c->upload(wid.data(), ns);
    F.ci = c->upload(ci.data(), slots);
    if (M.f32) {
        std::vector<float> f(val.begin(), val.end());
        F.v32 = c->upload(f.data(), static_cast<int64_t>(f.size()));
    } else {
        F.v64 = c->upload(val.data(), static_cast<int64_t>(val.size()));
    }
    F.slots = slots;
    F.G = G;
}

// New values of every sliced form of M from its device CSR values (FP64).
static void refresh_sells(msp_ctx* c, DevCsr& M, hipStream_t st) {
    for (int q = 0; q < kSellForms; ++q) {
        DevSell& F = M.sell[q];
        if (!F.G) continue;
        if (!F.pos) {
            std::vector<int64_t> off, pos;
            std::vector<int32_t> wid;
            sell_layout(*M.hpat, F.G, off, wid, pos);
            F.pos = c->upload(pos.data(), static_cast<int64_t>(pos.size()));
        }
        HIPCHECK(launch_sell_values(st, F.slots, M.vs, F.pos, M.v64, M.f32 ? nullptr : F.v64, M.f32 ? F.v32 : nullptr));
    }
}

static void free_sell(msp_ctx* c, DevSell& F) {
    for (void* q : {static_cast<void*>(F.off), static_cast<void*>(F.wid), static_cast<void*>(F.ci),
                    static_cast<void*>(F.v64), static_cast<void*>(F.v32), static_cast<void*>(F.pos)})
        if (q) c->dfree(q);
    F = DevSell();
}


// Key of one tuned choice in a tuning file: precision, preconditioner, base
// rows, level, matrix, multivector type and column count.
static std::string tune_key(const msp_ctx* c, size_t l, const char* what, int ts, int C) {
    return "p" + std::to_string(c->o.precision) + " pc" + std::to_string(c->o.pc) + " nb" +
           std::to_string(c->sym.n_b) + " L" + std::to_string(l) + " " + what + " t" + std::to_string(ts) + " c" +
           std::to_string(C);
}

// Autotuner: for every V-cycle matrix and this column count, time the
// candidate kernels -- the CSR kernels with 1, 2, 4, ... lane groups per row
// (up to the block's capacity and about half the mean row length), their
// 16-byte-lane form, and the sliced-ELL kernel with rows split G = 1, 2, 4,
// ... ways -- and keep the fastest.  Each candidate is timed as the solve
// sees it: the memory-side cache is first cleared by writing a 512 MB block,
// the input multivector is rewritten (in the solve it was just produced),
// then the product alone runs between two events; the median of three such
// runs counts.  Runs once per context and column count.
// Fixed variants instead of timings (every variant computes the same
// product; tests use these to cover each one): MSP_SPMM_SPLIT=g (a power of
// two; clamped to what a block holds), MSP_SPMM_WIDE=1 (16-byte lanes where a
// matrix has them), MSP_SPMM_SELL=G (the sliced-ELL kernel with the largest
// row split <= G that fits; 0 = the CSR kernels), MSP_DENSE_ROWS=R (1, 2, 4
// or 8 rows per wavefront).  MSP_TUNE_SAVE=path appends the choices to a
// file, MSP_TUNE_LOAD=path takes them from one (a profiler run then launches
// the kernels a timed run chose).
template <typename T>
static void autotune_level_splits(msp_ctx* c, Work& w) {
    hipStream_t st = nullptr;
    const int C = w.C;
    const int ts = tslot<T>(), lc = log2i(C);
    const int eb = static_cast<int>(sizeof(T));
    const int vw = lane_width(eb);
    const int lpr = C >= vw ? C / vw : 1;   // lanes per row of Lanes<T, C>
    const int S = 1 << c->sym.s;
    const int mt = std::max(1, C / S);   // columns per subsystem assumed for matrices with value sets
    const char* logv = std::getenv("MSP_AUTOTUNE_LOG");   // set (non-empty, not "0"): timings to stderr
    const bool log = logv && *logv && std::strcmp(logv, "0") != 0;
    static const char* const names[6] = {"A", "M", "R", "P", "G", "GT"};
    auto mats = [](DevLevel& L) { return std::array<DevCsr*, 6>{&L.A, &L.M, &L.R, &L.P, &L.G, &L.GT}; };
    auto sell_ok = [&](const DevCsr* M, int G, bool wide) {
        return M->hpat && !M->v16 && sell_fits(C, eb, G, wide && M->vs == 1);
    };
    const int force_split = env_int("MSP_SPMM_SPLIT");
    const int force_wide = env_int("MSP_SPMM_WIDE");
    const int force_sell = env_int("MSP_SPMM_SELL");
    const int force_rows = env_int("MSP_DENSE_ROWS");
    if (force_split > 0 || force_wide >= 0 || force_sell >= 0 || force_rows > 0) {
        int g = 1;
        while (force_split > 0 && g * 2 <= force_split && g * 2 * lpr <= 256) g *= 2;
        for (auto& L : c->dl)
            for (DevCsr* M : mats(L)) {
                M->tuned[ts][lc] = g;
                const bool wd = force_wide == 1 && M->vs == 1 && spmm_has_wide(C, eb);
                M->wide[ts][lc] = (g == 1 || force_sell > 0) && wd;
                int G = 0;
                if (force_sell > 0 && M->nnz > 0) {
                    G = 1;
                    while (G * 2 <= force_sell && sell_ok(M, G * 2, wd)) G *= 2;
                    if (!sell_ok(M, G, wd)) G = 0;
                    if (G) build_sell(c, *M, G);
                }
                M->sg[ts][lc] = G;
            }
        int R = 1;
        while (force_rows > 0 && R * 2 <= force_rows && R * 2 <= 8) R *= 2;
        w.dense_rows = force_rows > 0 ? R : 8;
        return;
    }
    // choices from a tuning file, when it has every one of them
    if (const char* path = std::getenv("MSP_TUNE_LOAD")) {
        std::map<std::string, std::array<int, 3>> tab;
        if (std::FILE* f = std::fopen(path, "r")) {
            char line[512];
            while (std::fgets(line, sizeof(line), f)) {
                std::string ln(line);
                const size_t eq = ln.find('=');
                if (eq == std::string::npos) continue;
                std::array<int, 3> v{0, 0, 0};
                if (std::sscanf(ln.c_str() + eq + 1, "%d %d %d", &v[0], &v[1], &v[2]) >= 1) tab[ln.substr(0, eq)] = v;
            }
            std::fclose(f);
        }
        bool all = true;
        for (size_t l = 0; l < c->dl.size() && all; ++l) {
            auto ms = mats(c->dl[l]);
            for (int j = 0; j < 6 && all; ++j)
                if (ms[j]->nnz) all = tab.count(tune_key(c, l, names[j], ts, C)) > 0;
        }
        const std::string dk = tune_key(c, c->dl.size(), "dense", ts, C);
        if (c->sub) all = all && tab.count(dk);
        if (all) {
            for (size_t l = 0; l < c->dl.size(); ++l) {
                auto ms = mats(c->dl[l]);
                for (int j = 0; j < 6; ++j) {
                    if (!ms[j]->nnz) continue;
                    const auto& v = tab[tune_key(c, l, names[j], ts, C)];
                    ms[j]->tuned[ts][lc] = std::max(1, v[0]);
                    ms[j]->wide[ts][lc] = v[1] != 0;
                    ms[j]->sg[ts][lc] = v[2];
                    if (v[2] > 0) build_sell(c, *ms[j], v[2]);
                }
            }
            if (c->sub) w.dense_rows = tab[dk][0];
            return;
        }
    }
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    const int64_t flush_n = int64_t(1) << 27;   // 512 MB of int: more than the memory-side cache
    int* flush = c->dalloc<int>(flush_n);
    for (size_t l = 0; l < c->hier.lev.size(); ++l) {
        const int64_t n = c->hier.lev[l].A.nr;
        HIPCHECK(launch_fill<T>(st, n * C, static_cast<T*>(w.vy[l]), T{}));
        HIPCHECK(launch_fill<T>(st, n * C, static_cast<T*>(w.vs[l]), T{}));
        HIPCHECK(launch_fill<T>(st, n * C, static_cast<T*>(w.vr[l]), T{}));
    }
    // median of three runs of launch(), each after the cache is cleared and X rewritten
    auto time_cold = [&](const T* X, int64_t nx, auto&& launch) {
        float t[3];
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHECK(launch_fill<int>(st, flush_n, flush, rep));
            HIPCHECK(launch_fill<T>(st, nx * C, const_cast<T*>(X), T{}));
            HIPCHECK(hipEventRecord(e0, st));
            launch();
            HIPCHECK(hipEventRecord(e1, st));
            HIPCHECK(hipEventSynchronize(e1));
            HIPCHECK(hipEventElapsedTime(&t[rep], e0, e1));
        }
        std::sort(t, t + 3);
        return t[1];
    };
    std::string saved;
    for (size_t l = 0; l < c->dl.size(); ++l) {
        DevLevel& L = c->dl[l];
        struct Job { DevCsr* M; const T* X; T* Y; };
        T* vs = static_cast<T*>(w.vs[l]);
        T* vr = static_cast<T*>(w.vr[l]);
        T* vt = w.vt[l] ? static_cast<T*>(w.vt[l]) : vr;
        Job jobs[6] = {{&L.A, vs, vr}, {&L.M, vr, vs}, {&L.R, vr, static_cast<T*>(w.vy[l + 1])},
                       {&L.P, static_cast<T*>(w.vs[l + 1]), vs}, {&L.G, vr, vt}, {&L.GT, vt, vs}};
        for (int j = 0; j < 6; ++j) {
            Job& jb = jobs[j];
            if (jb.M->nnz == 0) continue;
            const double avg = jb.M->nr ? static_cast<double>(jb.M->nnz) / static_cast<double>(jb.M->nr) : 0.0;
            struct Cand { int g; bool wide; int sg; };
            std::vector<Cand> cand;
            for (int g = 1; g <= 64 && g * lpr <= 256; g *= 2) {   // 256 threads per block
                if (g > 1 && g > std::max(1.0, avg / 2.0)) break;
                cand.push_back({g, false, 0});
                if (g == 1 && jb.M->vs == 1 && spmm_has_wide(C, eb)) cand.push_back({1, true, 0});
            }
            for (int G = 1; G <= 16; G *= 2) {
                if (G > 1 && G > std::max(1.0, avg / 2.0)) break;
                if (sell_ok(jb.M, G, false)) cand.push_back({1, false, G});
                if (jb.M->vs == 1 && spmm_has_wide(C, eb) && sell_ok(jb.M, G, true)) cand.push_back({1, true, G});
            }
            Cand best = cand[0];
            float best_ms = 1e30f;
            for (const Cand& cd : cand) {
                if (cd.sg > 0) build_sell(c, *jb.M, cd.sg);
                const int64_t nx = jb.M->nc;
                auto run = [&] {
                    spmm_launch<T>(st, C, *jb.M, cd.g, cd.wide, jb.X, jb.Y, nullptr, acc_t<T>(1), acc_t<T>(0),
                                   OuterDiag{nullptr, nullptr}, S, mt, cd.sg);
                };
                run();   // first launch of this kernel shape (code load) outside the timing
                const float ms = time_cold(jb.X, nx, run);
                if (log)
                    std::fprintf(stderr, "msp autotune: C=%d elem=%d level %zu %s (%lld rows, %.1f nnz/row, %d sets) "
                                 "%s %d%s: %.2f us\n", C, eb, l, names[j], static_cast<long long>(jb.M->nr), avg,
                                 jb.M->vs, cd.sg ? "sliced G" : "split", cd.sg ? cd.sg : cd.g,
                                 cd.wide ? " wide" : "", 1000.0 * ms);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = cd;
                }
            }
            jb.M->tuned[ts][lc] = best.g;
            jb.M->wide[ts][lc] = best.wide;
            jb.M->sg[ts][lc] = best.sg;
            saved += tune_key(c, l, names[j], ts, C) + "=" + std::to_string(best.g) + " " +
                     std::to_string(best.wide ? 1 : 0) + " " + std::to_string(best.sg) + "\n";
            // drop the sliced forms no column count uses
            for (int q = 0; q < kSellForms; ++q) {
                DevSell& F = jb.M->sell[q];
                if (!F.G) continue;
                bool used = false;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 7; ++b) used |= jb.M->tuned[a][b] && jb.M->sg[a][b] == F.G;
                if (!used) free_sell(c, F);
            }
        }
    }
    // rows per wavefront of the per-subsystem coarsest solves
    if (c->sub) {
        const size_t Lc = c->hier.lev.size() - 1;
        T* y = static_cast<T*>(w.vy[Lc]);
        T* s = static_cast<T*>(w.vs[Lc]);
        float best_ms = 1e30f;
        for (int R = 1; R <= dense_sets_rows_max(mt); R *= 2) {
            auto run = [&] { dense_sets<T>(c, w, st, mt, y, s, R); };
            run();
            const float ms = time_cold(y, c->nL, run);
            if (log)
                std::fprintf(stderr, "msp autotune: C=%d elem=%d coarsest solves, %d rows per wavefront: %.2f us\n", C,
                             eb, R, 1000.0 * ms);
            if (ms < best_ms) {
                best_ms = ms;
                w.dense_rows = R;
            }
        }
        saved += tune_key(c, Lc, "dense", ts, C) + "=" + std::to_string(w.dense_rows) + "\n";
    }
    HIPCHECK(hipStreamSynchronize(st));
    c->dfree(flush);
    HIPCHECK(hipEventDestroy(e0));
    HIPCHECK(hipEventDestroy(e1));
    if (const char* path = std::getenv("MSP_TUNE_SAVE")) {
        if (std::FILE* f = std::fopen(path, "a")) {
            std::fputs(saved.c_str(), f);
            std::fclose(f);
        }
    }
}

// The operator kernel (A_inn + outer diagonal, FP64) on its CSR or its
// sliced-ELL form: both timed once per column count in the same cold-cache
// conditions as the V-cycle products, the faster kept.  MSP_OP_SELL=0/1
// fixes the choice; MSP_TUNE_LOAD / MSP_TUNE_SAVE as for the V-cycle.
static void autotune_operator(msp_ctx* c, Work& w) {
    const int C = w.C, lc = log2i(C);
    const int S = 1 << c->sym.s;
    const int64_t nb = c->sym.n_b;
    const std::string key = tune_key(c, 0, "op", 0, C);
    int choice = env_int("MSP_OP_SELL");
    if (choice < 0) {
        if (const char* path = std::getenv("MSP_TUNE_LOAD")) {
            if (std::FILE* f = std::fopen(path, "r")) {
                char line[512];
                while (std::fgets(line, sizeof(line), f)) {
                    const std::string ln(line);
                    const size_t eq = ln.find('=');
                    if (eq != std::string::npos && ln.substr(0, eq) == key) choice = std::atoi(ln.c_str() + eq + 1);
                }
                std::fclose(f);
            }
        }
    }
    if (choice >= 0) {
        if (choice > 0) build_sell(c, c->dAinn, 1);
        c->op_sell[lc] = choice > 0 ? 1 : 0;
        return;
    }
    build_sell(c, c->dAinn, 1);
    hipStream_t st = nullptr;
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    const int64_t flush_n = int64_t(1) << 27;   // 512 MB of int: more than the memory-side cache
    int* flush = c->dalloc<int>(flush_n);
    const DevSell& F = c->dAinn.sell[0];
    float best = 1e30f;
    int pick = 0;
    for (int v = 0; v < 2; ++v) {
        const SellRef sl = v ? SellRef{F.off, F.wid, F.ci, F.v64} : SellRef{nullptr, nullptr, nullptr, nullptr};
        int grid = 0;
        HIPCHECK(op_dot_grid(C, v == 1, nb, &grid));
        auto run = [&] {
            HIPCHECK(launch_op_dot(st, C, grid, nb, c->dAinn.rp, c->dAinn.ci, c->dAinn.v64, sl, c->dsig.d, S, 1, w.p,
                                   w.q, w.pp1));
        };
        HIPCHECK(launch_fill<double>(st, nb * C, w.p, 0.0));
        run();
        float t[3];
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHECK(launch_fill<int>(st, flush_n, flush, rep));
            HIPCHECK(launch_fill<double>(st, nb * C, w.p, 0.0));
            HIPCHECK(hipEventRecord(e0, st));
            run();
            HIPCHECK(hipEventRecord(e1, st));
            HIPCHECK(hipEventSynchronize(e1));
            HIPCHECK(hipEventElapsedTime(&t[rep], e0, e1));
        }
        std::sort(t, t + 3);
        const char* logv = std::getenv("MSP_AUTOTUNE_LOG");
        if (logv && *logv && std::strcmp(logv, "0") != 0)
            std::fprintf(stderr, "msp autotune: C=%d operator %s: %.2f us\n", C, v ? "sliced" : "CSR", 1000.0 * t[1]);
        if (t[1] < best) {
            best = t[1];
            pick = v;
        }
    }
    c->op_sell[lc] = pick;
    HIPCHECK(hipStreamSynchronize(st));
    c->dfree(flush);
    HIPCHECK(hipEventDestroy(e0));
    HIPCHECK(hipEventDestroy(e1));
    if (const char* path = std::getenv("MSP_TUNE_SAVE")) {
        if (std::FILE* f = std::fopen(path, "a")) {
            std::fprintf(f, "%s=%d\n", key.c_str(), pick);
            std::fclose(f);
        }
    }
}

// bytes per element of the V-cycle multivectors
static int vbytes(const msp_ctx* c) {
    return c->o.precision == MSP_FP64 ? 8 : (c->o.precision == MSP_MIXED_BF16 ? 2 : 4);
}
static bool amg(const msp_ctx* c) { return c->o.pc == MSP_PC_AMGR || c->o.pc == MSP_PC_AMGR_SUB; }
static bool amgs(const msp_ctx* c) { return c->o.pc == MSP_PC_AMGS; }
// a multigrid hierarchy is uploaded and cycled: A_inn's (AMGR) or K's (AMGS)
static bool cycle(const msp_ctx* c) { return amg(c) || amgs(c); }

// Carves the device arrays of a C-column workspace out of base (base ==
// nullptr: offsets only); each array starts on a 256-byte boundary.  Returns
// the bytes the block needs.
static size_t carve_work(const msp_ctx* c, int C, Work& w, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        off = (off + 255) & ~static_cast<size_t>(255);
        void* p = base ? static_cast<void*>(base + off) : nullptr;
        off += bytes > 0 ? bytes : 1;
        return p;
    };
    const size_t nb = static_cast<size_t>(c->sym.n_b);
    const size_t vec = sizeof(double) * nb * static_cast<size_t>(C);
    w.C = C;
    w.x = static_cast<double*>(take(vec));
    w.r = static_cast<double*>(take(vec));
    w.z = static_cast<double*>(take(vec));
    w.p = static_cast<double*>(take(vec));
    w.q = static_cast<double*>(take(vec));
    w.zold = static_cast<double*>(take(vec));
    if (amgs(c)) {
        w.amgs1 = static_cast<double*>(take(vec));
        w.amgs2 = static_cast<double*>(take(vec));
    }
    const size_t es = static_cast<size_t>(vbytes(c));
    const size_t L = c->hier.lev.size();
    if (cycle(c)) {
        for (size_t l = 0; l < L; ++l) {
            const size_t n = static_cast<size_t>(c->hier.lev[l].A.nr);
            w.vy[l] = take(es * n * C);
            w.vs[l] = take(es * n * C);
            w.vr[l] = take(es * n * C);
            if (c->o.precision == MSP_MIXED_FP32_BF16G) w.vt[l] = take(es * n * C);
        }
        const int64_t nL = c->hier.lev.back().A.nr;
        const int ks = dense_splits(C, nL, vbytes(c));
        w.dense_part = static_cast<double*>(take(sizeof(double) * static_cast<size_t>(ks * nL * C)));
        if (c->sub) w.dense_pack = take(sizeof(double) * static_cast<size_t>(2 * (nL + 4) * C));
    }
    w.nb_dot = 512;
    w.partial = static_cast<double*>(take(sizeof(double) * static_cast<size_t>(w.nb_dot) * 64));
    w.pp1 = static_cast<double*>(take(sizeof(double) * static_cast<size_t>(kPcgMaxBlocks) * 64));
    w.pp2 = static_cast<double*>(take(sizeof(double) * static_cast<size_t>(kPcgMaxBlocks) * 64));
    if (c->lrc_k > 0)
        w.plrc = static_cast<double*>(take(sizeof(double) * static_cast<size_t>(kPcgMaxBlocks) * 64 * c->lrc_k));
    w.scal = static_cast<double*>(take(sizeof(double) * SC_COUNT * 64));
    w.iscal = static_cast<int*>(take(sizeof(int) * (64 * 2 + 2)));
    return off;
}

// Pinned host buffers for the flags and statistics of a solve.
static void alloc_host_bufs(HostBufs& h) {
    HIPCHECK(hipHostMalloc(reinterpret_cast<void**>(&h.h_flags), 2 * sizeof(int), hipHostMallocDefault));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void**>(&h.h_pub), 4 * sizeof(int),
                           hipHostMallocMapped | hipHostMallocCoherent));
    h.h_pub[0] = h.h_pub[1] = h.h_pub[2] = h.h_pub[3] = 0;
    HIPCHECK(hipHostGetDevicePointer(reinterpret_cast<void**>(&h.d_pub), h.h_pub, 0));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void**>(&h.h_iters), 64 * sizeof(int), hipHostMallocDefault));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void**>(&h.h_scal), SC_COUNT * 64 * sizeof(double),
                           hipHostMallocDefault));
}

static void use_host_bufs(Work& w, const HostBufs& h) {
    w.h_flags = h.h_flags;
    w.h_pub = h.h_pub;
    w.d_pub = h.d_pub;
    w.h_iters = h.h_iters;
    w.h_scal = h.h_scal;
}

// Workspace for C padded columns (allocated on first use, kept with the context).
static Work& work(msp_ctx* c, int C) {
    auto it = c->works.find(C);
    if (it != c->works.end()) return *it->second;
    std::unique_ptr<Work> wp(new Work());
    Work& w = *wp;
    const size_t bytes = carve_work(c, C, w, nullptr);
    carve_work(c, C, w, c->dalloc<char>(static_cast<int64_t>(bytes)));
    alloc_host_bufs(w.own);
    use_host_bufs(w, w.own);
    c->works[C] = std::move(wp);
    autotune_operator(c, w);
    if (cycle(c) && !c->dl.empty()) {
        if (c->o.precision == MSP_MIXED_BF16) autotune_level_splits<Bf16>(c, w);
        else if (mixed(c)) autotune_level_splits<float>(c, w);
        else autotune_level_splits<double>(c, w);
    }
    return w;
}

// One V(1,1) cycle of Alg. 3 on level l: s = M_l^{-1} y, all C columns.
template <typename T>
static void vcycle(msp_ctx* c, Work& w, hipStream_t st, size_t l, const T* y, T* s) {
    const int C = w.C;
    const int S = 1 << c->sym.s;
    if (l + 1 == c->hier.lev.size()) {
        if (c->sub && l > 0) {   // every subsystem's own coarsest operator
            timed(c, KD_DENSE, dense_sets_bytes<T>(c, C), st, [&] { dense_sets<T>(c, w, st, w.m, y, s, w.dense_rows); },
                  [&] {
                      int mp = 1;
                      while (mp < w.m) mp *= 2;
                      return std::string("k_pack_sets+k_dense_sets<") + tname<T>() + ", " +
                             (std::is_same<T, double>::value || !c->d_cinv32 ? "double" : "float") + ", " +
                             std::to_string(mp) + ", " + std::to_string(w.dense_rows) + ">";
                  });
        } else {
            const double bytes = 8.0 * c->nL * c->nL + 2.0 * sizeof(T) * c->nL * C;
            timed(c, KD_DENSE, bytes, st,
                  [&] { HIPCHECK(launch_dense<T>(st, C, c->nL, c->d_cinv, y, s, w.dense_part, c->gate)); },
                  [&] { return std::string("k_dense_part+k_dense_sum<") + tname<T>() + ", " + std::to_string(C) + ">"; });
        }
        return;
    }
    const DevLevel& L = c->dl[l];
    T* r = static_cast<T*>(w.vr[l]);
    T* yc = static_cast<T*>(w.vy[l + 1]);
    T* sc = static_cast<T*>(w.vs[l + 1]);
    const int kb = KD_LEVEL + 8 * static_cast<int>(l);
    // smoother s = beta s + M v with M = w G^T G (explicit, or factored with a temporary)
    using TC = acc_t<T>;
    auto smooth = [&](const T* v, TC beta) {
        if (L.G.nnz) {
            T* t = static_cast<T*>(w.vt[l]);
            spmm<T>(c, kb + 1, st, C, L.G, v, t, nullptr, TC(1), TC(0));
            spmm<T>(c, kb + 2, st, C, L.GT, t, s, beta != TC(0) ? s : nullptr, static_cast<TC>(L.omega), beta);
        } else {
            spmm<T>(c, kb + 1, st, C, L.M, v, s, beta != TC(0) ? s : nullptr, TC(1), beta, nullptr, 1 << c->sym.s,
                    w.m);
        }
    };
    // per-subsystem hierarchy: the reduction level applies each subsystem's
    // operator A_inn + diag(sigma_a); the levels below carry one value set per subsystem
    const DevOuter* sg = !c->sub ? nullptr : (l == 0 ? &c->dsig : (l == 1 ? &c->dsig1 : nullptr));
    const int m = w.m;
    smooth(y, TC(0));                                                      // pre-smooth from zero: s = M y
    for (int i = 1; i < c->o.nu1; ++i) {                                   // further sweeps s += M (y - A s)
        spmm<T>(c, kb + 0, st, C, L.A, s, r, y, TC(-1), TC(1), sg, S, m);
        smooth(r, TC(1));
    }
    spmm<T>(c, kb + 0, st, C, L.A, s, r, y, TC(-1), TC(1), sg, S, m);      // r = y - A s
    spmm<T>(c, kb + 3, st, C, L.R, r, yc, nullptr, TC(1), TC(0), nullptr, S, m);   // r_c = P^T r
    vcycle<T>(c, w, st, l + 1, yc, sc);                                    // coarse correction
    spmm<T>(c, kb + 4, st, C, L.P, sc, s, s, TC(1), TC(1), nullptr, S, m);  // s += P h_c
    for (int i = 0; i < c->o.nu2; ++i) {                                   // post-smooth: s += M (y - A s)
        spmm<T>(c, kb + 0, st, C, L.A, s, r, y, TC(-1), TC(1), sg, S, m);
        smooth(r, TC(1));
    }
}

// out[c] = <X_c, Y_c> for the C columns of two rows x C multivectors (rows = n_b by default).
static void dot(msp_ctx* c, Work& w, hipStream_t st, const double* X, const double* Y, double* out,
                int64_t rows = -1) {
    const int64_t nb = rows >= 0 ? rows : c->sym.n_b;
    const int C = w.C;
    timed(c, KD_DOT, 16.0 * nb * C, st,
          [&] { HIPCHECK(launch_dot<double>(st, C, nb, X, Y, w.partial, w.nb_dot, out)); },
          [&] { return "k_dot+k_reduce_partials<double, " + std::to_string(C) + ">"; });
}

// z += U_a diag(coef_a) U_a^T r_a for every subsystem a (low-rank corrections).
static void lrc_apply(msp_ctx* c, Work& w, hipStream_t st, const double* r, double* z, int64_t rows = -1) {
    const int64_t nb = rows >= 0 ? rows : c->sym.n_b;
    const int S = 1 << c->sym.s, k = c->lrc_k;
    const double bytes = 2.0 * nb * S * k * (c->U32 ? 4.0 : 8.0) + 3.0 * 8.0 * nb * w.C;
    timed(c, KD_LRC, bytes, st, [&] {
        if (c->U32)
            HIPCHECK(launch_lrc_apply<float>(st, nb, S, k, w.m, w.C, static_cast<const float*>(c->d_U), r, z,
                                             c->d_lrc_coef, c->d_lrc_part, c->lrc_nb, c->d_lrc_W));
        else
            HIPCHECK(launch_lrc_apply<double>(st, nb, S, k, w.m, w.C, static_cast<const double*>(c->d_U), r, z,
                                              c->d_lrc_coef, c->d_lrc_part, c->lrc_nb, c->d_lrc_W));
    }, [] { return std::string("k_lrc_project+k_lrc_finish+k_lrc_expand"); });
}

// The shared preconditioner without corrections: the V-cycle (AMGR), G^T G
// (FSAI) or the identity.  For FSAI with corrections the correction acts on
// t = G r before the G^T product: z = G^T (t + V Theta V^T t).
static void precondition_base(msp_ctx* c, Work& w, hipStream_t st, const double* r, double* z,
                              bool with_lrc_fsai) {
    const int C = w.C;
    const int64_t nb = c->sym.n_b;
    if (amg(c)) {
        if (mixed(c)) {
            auto run = [&](auto tag) {
                using T = decltype(tag);
                T* y0 = static_cast<T*>(w.vy[0]);
                T* s0 = static_cast<T*>(w.vs[0]);
                const double cb = (8.0 + sizeof(T)) * nb * C;
                timed(c, KD_CAST, cb, st, [&] { HIPCHECK((launch_cast<T, double>(st, nb * C, r, y0))); },
                      [] { return std::string("k_cast<") + tname<T>() + ", double>"; });
                vcycle<T>(c, w, st, 0, y0, s0);
                timed(c, KD_CAST, cb, st, [&] { HIPCHECK((launch_cast<double, T>(st, nb * C, s0, z))); },
                      [] { return std::string("k_cast<double, ") + tname<T>() + ">"; });
            };
            if (c->o.precision == MSP_MIXED_BF16) run(Bf16{});
            else run(0.0f);
        } else {
            vcycle<double>(c, w, st, 0, r, z);
        }
    } else if (amgs(c)) {
        // eq. (3.12) with base cells ordered inner first: r = [r_I; r_G], z = [z_I; z_G]
        const int64_t nI = c->am.nI, nG = nb - nI;
        const double* rI = r;
        const double* rG = r + nI * C;
        double* zI = z;
        double* zG = z + nI * C;
        vcycle<double>(c, w, st, 0, rI, zI);                                         // t = AMG_K r_I (in z_I)
        spmm<double>(c, KD_AMGS, st, C, c->dBT, zI, w.amgs1, rG, -1.0, 1.0);        // q = r_G - B^T t
        spmm<double>(c, KD_AMGS, st, C, c->dGS1, w.amgs1, w.amgs2, nullptr, 1.0, 0.0);   // u = G_S1 q
        if (c->d_U) {                                                                // u += V Theta V^T u
            HIPCHECK(hipMemcpyAsync(w.amgs1, w.amgs2, sizeof(double) * nG * C, hipMemcpyDeviceToDevice, st));
            lrc_apply(c, w, st, w.amgs1, w.amgs2, nG);
        }
        spmm<double>(c, KD_AMGS, st, C, c->dGS1T, w.amgs2, zG, nullptr, 1.0, 0.0);   // z_G = G_S1^T u
        spmm<double>(c, KD_AMGS, st, C, c->dB, zG, w.amgs1, nullptr, 1.0, 0.0);     // v = B z_G
        if (c->o.amgs_light) {                                                       // z_I = t - G_K^T G_K v
            spmm<double>(c, KD_AMGS, st, C, c->dGK, w.amgs1, w.amgs2, nullptr, 1.0, 0.0);
            spmm<double>(c, KD_AMGS, st, C, c->dGKT, w.amgs2, zI, zI, -1.0, 1.0);
        } else {                                                                     // z_I = t - AMG_K v
            vcycle<double>(c, w, st, 0, w.amgs1, w.amgs2);
            HIPCHECK(launch_axpy_cols(st, nI * C, C, zI, w.amgs2, c->d_ones));
        }
    } else if (c->o.pc == MSP_PC_FSAI) {
        double* t = w.zold;   // scratch (the FSAI mode keeps no flexible copy)
        spmm<double>(c, KD_FSAI, st, C, c->dGf, r, t, nullptr, 1.0, 0.0);
        if (with_lrc_fsai && c->d_U) {
            // t += V Theta V^T t: apply in place through a copy of t held in z
            HIPCHECK(hipMemcpyAsync(z, t, sizeof(double) * nb * C, hipMemcpyDeviceToDevice, st));
            lrc_apply(c, w, st, z, t);
        }
        spmm<double>(c, KD_FSAI, st, C, c->dGfT, t, z, nullptr, 1.0, 0.0);
    } else {
        HIPCHECK(hipMemcpyAsync(z, r, sizeof(double) * nb * C, hipMemcpyDeviceToDevice, st));
    }
}

// Compact outer diagonal: rows whose S values are not all zero, in row order.
static DevOuter upload_outer(msp_ctx* c, const std::vector<double>& dense, int64_t rows, int S) {
    std::vector<int32_t> idx(rows, -1);
    std::vector<double> val;
    int32_t q = 0;
    for (int64_t i = 0; i < rows; ++i) {
        bool any = false;
        for (int a = 0; a < S; ++a) any |= dense[i * S + a] != 0.0;
        if (!any) continue;
        idx[i] = q++;
        val.insert(val.end(), dense.begin() + i * S, dense.begin() + (i + 1) * S);
    }
    DevOuter o;
    o.rows = rows;
    o.carried = q;
    o.d.idx = c->upload(idx.data(), rows);
    o.d.val = c->upload(val.data(), static_cast<int64_t>(val.size()));
    return o;
}

static void upload_all(msp_ctx* c) {
    HIPCHECK(hipSetDevice(c->device));
    const bool f32 = mixed(c);
    c->d_img = c->upload(c->sym.img.data(), static_cast<int64_t>(c->sym.img.size()));
    c->dsig = upload_outer(c, c->sym.sigma, c->sym.n_b, 1 << c->sym.s);
    c->dAinn = upload_csr(c, c->sym.Ainn, false);
    c->dAinn.hpat = &c->sym.Ainn;   // the operator's sliced form is built from these (FP64 values)
    c->dAinn.hval = &c->sym.Ainn.v;
    if (cycle(c)) {
        const int S = 1 << c->sym.s;
        c->dl.resize(c->hier.lev.size() - 1);
        for (size_t l = 0; l + 1 < c->hier.lev.size(); ++l) {
            const HostLevel& H = c->hier.lev[l];
            DevLevel& D = c->dl[l];
            D.n = H.A.nr;
            D.omega = H.omega;
            auto keep_host = [&](DevCsr& Dm, const Csr& pat, const std::vector<double>& val) {
                Dm.hpat = &pat;
                Dm.hval = &val;
                Dm.f32 = f32;
            };
            if (c->sub && l > 0) {
                // one value set per subsystem on the shared patterns; the smoother is
                // explicit (omega_a G_a^T G_a) in every precision.  A_1,a = A_1 + diag(sigma_a)
                // on the coarse interface points, so level 1 keeps the shared values and
                // applies the outer diagonal like the reduction level does.
                if (l == 1) {
                    D.A = upload_csr(c, H.A, f32);
                    keep_host(D.A, H.A, H.A.v);
                    std::vector<double> s1(static_cast<size_t>(H.A.nr) * S, 0.0);
                    int64_t j = 0;
                    const HostLevel& L0 = c->hier.lev[0];
                    for (int64_t i = 0; i < L0.A.nr; ++i) {
                        if (!L0.cf[i]) continue;
                        if (c->sym.iface[i])
                            for (int a = 0; a < S; ++a) s1[j * S + a] = c->sym.sigma[i * S + a];
                        ++j;
                    }
                    if (j != H.A.nr) throw Error(MSP_ERR_ARG, "coarse numbering of the reduction level");
                    c->dsig1 = upload_outer(c, s1, H.A.nr, S);
                } else {
                    D.A = upload_sets(c, H.A, c->subv.A[l], S, f32);
                    keep_host(D.A, H.A, c->subv.A[l]);
                }
                D.P = upload_sets(c, H.P, c->subv.P[l], S, f32);
                D.R = upload_sets(c, H.R, c->subv.R[l], S, f32);
                D.M = upload_sets(c, H.M, c->subv.M[l], S, f32);
                keep_host(D.P, H.P, c->subv.P[l]);
                keep_host(D.R, H.R, c->subv.R[l]);
                keep_host(D.M, H.M, c->subv.M[l]);
                continue;
            }
            D.A = upload_csr(c, H.A, f32);
            D.P = upload_csr(c, H.P, f32);
            D.R = upload_csr(c, H.R, f32);
            keep_host(D.A, H.A, H.A.v);
            keep_host(D.P, H.P, H.P.v);
            keep_host(D.R, H.R, H.R.v);
            if (c->o.precision == MSP_MIXED_FP32_BF16G) {
                // the smoother is kept factored, G^T (G r) with bfloat16 factors, so it stays SPD;
                // its damping is recomputed for the rounded factors (rounding can raise
                // lambda_max(G A G^T) where large terms cancel)
                D.G = upload_csr(c, H.G, true, true);
                D.GT = upload_csr(c, H.GT, true, true);
                Csr Gr = H.G, GTr = H.GT;
                for (double& v : Gr.v) v = bf16_value(v);
                for (double& v : GTr.v) v = bf16_value(v);
                D.omega = damping(H.A, Gr, GTr, c->o.seed);
            } else {
                D.M = upload_csr(c, H.M, f32);
                keep_host(D.M, H.M, H.M.v);
            }
        }
        c->nL = c->hier.lev.back().A.nr;
        const std::vector<double>& inv = c->sub ? c->subv.coarse_inv : c->hier.coarse_inv;
        if (c->sub && mixed(c) && !c->o.coarse64) {
            // the V-cycle computes in FP32: its coarsest inverses are read in FP32 too
            const int64_t nL = c->nL, ld = dense_sets_ld(nL, 4);
            const int64_t S = int64_t(1) << c->sym.s;
            std::vector<float> f(static_cast<size_t>(S * nL * ld), 0.0f);
            for (int64_t a = 0; a < S; ++a)
                for (int64_t i = 0; i < nL; ++i)
                    for (int64_t k = 0; k < nL; ++k)
                        f[static_cast<size_t>((a * nL + i) * ld + k)] =
                            static_cast<float>(inv[static_cast<size_t>((a * nL + i) * nL + k)]);
            c->d_cinv32 = c->upload(f.data(), static_cast<int64_t>(f.size()));
        } else {
            c->d_cinv = c->upload(inv.data(), static_cast<int64_t>(inv.size()));
        }
    } else if (c->o.pc == MSP_PC_FSAI) {
        c->dGf = upload_csr(c, c->Gf, false);
        c->dGfT = upload_csr(c, transpose(c->Gf), false);
    }
    if (amgs(c)) {
        const AmgsParts& A = c->am;
        c->dB = upload_csr(c, A.B, false);
        c->dBT = upload_csr(c, A.BT, false);
        c->dC1 = upload_csr(c, A.C1, false);
        c->dGK = upload_csr(c, A.GK, false);
        c->dGKT = upload_csr(c, A.GKT, false);
        c->dGS1 = upload_csr(c, A.GS1, false);
        c->dGS1T = upload_csr(c, A.GS1T, false);
        const int S = 1 << c->sym.s;
        const int64_t nG = c->sym.n_b - A.nI;
        std::vector<double> sg(c->sym.sigma.begin() + A.nI * S, c->sym.sigma.end());
        c->dsigG = upload_outer(c, sg, nG, S);
        std::vector<double> ones(64, 1.0);
        c->d_ones = c->upload(ones.data(), 64);
    }
    c->on_device = true;
}

static int next_pow2(int x) {
    int c = 1;
    while (c < x) c <<= 1;
    return c;
}

// One solve split into phases so that iterations can be enqueued without
// host synchronisation (and captured into a graph for batched solves):
//   begin:  norms, thresholds, Q_s forward, initial residual checks, z, rho, p
//   half_a: q = A p, alpha, x/r update, convergence check   (flags)
//   half_b: z = M^{-1} r (+ corrections), beta, p update
//   finish: Q_s backward, statistics
// Frozen columns are masked on the device (alpha = beta = 0), so extra
// iterations after convergence leave x unchanged.
struct SolvePlan {
    msp_ctx* c;
    Work* w;
    hipStream_t st;
    int m, S, C, kl, O;
    int nbo = 0, nbu = 0, nbz = 0;   // grids of the operator, update and z-finish kernels (partial rows)
    int nbp = 0;                     // grid of the rebuilding p update (mixed modes)
    const double* d_b0 = nullptr;    // the caller's right-hand sides (the true residual reads them again)
    bool vc_on = false;              // some V-cycle timer is on: t_vcycle_s is reported
    double vc_ms0 = 0.0;             // V-cycle timer total when this solve began
    int64_t nb, n;
    bool flexible, lrc_amg;
    bool x_pending = false;   // an x += alpha p step not yet applied
    double *rr, *rz, *pq, *rho, *alpha, *beta, *thr, *rnorm, *bn2;
    int *active, *iters, *flags;

    // noalloc: the workspace is carved from the device's static scratch array
    // (no allocation, no autotuning: the lane-group splits tuned by earlier
    // solves of this context and column count, else the defaults)
    SolvePlan(msp_ctx* c_, int m_, hipStream_t st_, Work* noalloc = nullptr) : c(c_), st(st_), m(m_) {
        if (!c->on_device) throw Error(MSP_ERR_ARG, "context was set up without a device");
        if (m <= 0) throw Error(MSP_ERR_ARG, "need m > 0");
        HIPCHECK(hipSetDevice(c->device));
        S = 1 << c->sym.s;
        const int ncol = S * m;
        if (ncol > 64) throw Error(MSP_ERR_UNSUPPORTED, "2^s * m must not exceed 64");
        C = next_pow2(ncol);
        if (noalloc) {
            char* base = static_cast<char*>(scratch_address(c->device));
            if (!base) throw Error(MSP_ERR_HIP, "scratch array not set up on this device");
            const size_t need = carve_work(c, C, *noalloc, nullptr);
            if (need > kScratchBytes)
                throw Error(MSP_ERR_UNSUPPORTED, "the allocation-free solve needs " + std::to_string(need) +
                                                     " bytes of workspace for this system and column count; the "
                                                     "scratch array holds " + std::to_string(kScratchBytes));
            carve_work(c, C, *noalloc, base);
            use_host_bufs(*noalloc, c->nohb);
            noalloc->pub_seq = c->nopub_seq;
            auto it = c->works.find(C);
            if (it != c->works.end()) noalloc->dense_rows = it->second->dense_rows;
            w = noalloc;
        } else {
            w = &work(c, C);
        }
        w->m = m;
        nb = c->sym.n_b;
        n = c->sym.n;
        double* sc = w->scal;
        rr = sc + SC_RR * 64; rz = sc + SC_RZ * 64; pq = sc + SC_PQ * 64; rho = sc + SC_RHO * 64;
        alpha = sc + SC_ALPHA * 64; beta = sc + SC_BETA * 64; thr = sc + SC_THR * 64;
        rnorm = sc + SC_RNORM * 64; bn2 = sc + SC_BN2 * 64;
        active = w->iscal;
        iters = w->iscal + 64;
        flags = w->iscal + 128;
        flexible = (mixed(c) && amg(c)) || (amgs(c) && c->o.amgs_light);
        lrc_amg = c->d_U && amg(c);
        kl = lrc_amg ? c->lrc_k : 0;
        O = S * kl * m;
        if (w->grid_op > 0) {   // the kernel variants are fixed per context and column count
            nbo = w->grid_op;
            nbu = w->grid_upd;
            nbz = w->grid_z;
            nbp = w->grid_p;
            return;
        }
        HIPCHECK(op_dot_grid(C, op_sliced(), nb, &nbo));
        if (c->U16) HIPCHECK(update_dots_grid<Bf16>(C, kl, nb, &nbu));
        else if (c->U32 || !c->d_U) HIPCHECK(update_dots_grid<float>(C, kl, nb, &nbu));
        else HIPCHECK(update_dots_grid<double>(C, kl, nb, &nbu));
        const bool lz = lrc_amg && kl > 0;
        const bool s16 = amg(c) && c->o.precision == MSP_MIXED_BF16, s32 = !s16 && amg(c) && mixed(c);
        if (s16) {
            if (c->U16) HIPCHECK((zfinish_grid<Bf16, Bf16>(C, lz, flexible, nb, &nbz)));
            else if (c->U32 || !c->d_U) HIPCHECK((zfinish_grid<Bf16, float>(C, lz, flexible, nb, &nbz)));
            else HIPCHECK((zfinish_grid<Bf16, double>(C, lz, flexible, nb, &nbz)));
            if (c->U16) HIPCHECK((pupdate_rebuild_grid<Bf16, Bf16>(C, lz, nb, &nbp)));
            else if (c->U32 || !c->d_U) HIPCHECK((pupdate_rebuild_grid<Bf16, float>(C, lz, nb, &nbp)));
            else HIPCHECK((pupdate_rebuild_grid<Bf16, double>(C, lz, nb, &nbp)));
        } else if (s32) {
            if (c->U32 || !c->d_U) HIPCHECK((zfinish_grid<float, float>(C, lz, flexible, nb, &nbz)));
            else HIPCHECK((zfinish_grid<float, double>(C, lz, flexible, nb, &nbz)));
            if (c->U32 || !c->d_U) HIPCHECK((pupdate_rebuild_grid<float, float>(C, lz, nb, &nbp)));
            else HIPCHECK((pupdate_rebuild_grid<float, double>(C, lz, nb, &nbp)));
        } else {
            if (c->U32 || !c->d_U) HIPCHECK((zfinish_grid<double, float>(C, lz, flexible, nb, &nbz)));
            else HIPCHECK((zfinish_grid<double, double>(C, lz, flexible, nb, &nbz)));
        }
        w->grid_op = nbo;
        w->grid_upd = nbu;
        w->grid_z = nbz;
        w->grid_p = nbp;
    }

    // the V-cycle's level-0 output in the mixed modes (z is rebuilt from it, not stored)
    const Bf16* cycle_out16() const {
        return (amg(c) && c->o.precision == MSP_MIXED_BF16) ? static_cast<const Bf16*>(w->vs[0]) : nullptr;
    }
    const float* cycle_out32() const {
        return (amg(c) && mixed(c) && c->o.precision != MSP_MIXED_BF16) ? static_cast<const float*>(w->vs[0])
                                                                         : nullptr;
    }

    double vb() const { return 8.0 * nb * C; }   // bytes of one FP64 multivector pass

    // the operator kernel on the sliced form (chosen by the first solve with this column count)
    bool op_sliced() const { return c->op_sell[log2i(C)] == 1 && c->dAinn.sell[0].G == 1; }
    SellRef op_sell_ref() const {
        const DevSell& F = c->dAinn.sell[0];
        return op_sliced() ? SellRef{F.off, F.wid, F.ci, F.v64} : SellRef{nullptr, nullptr, nullptr, nullptr};
    }
    double ubytes() const { return c->U16 ? 2.0 : (c->U32 ? 4.0 : 8.0); }   // bytes per element of U

    // the mixed AMGR mode writes the FP32 V-cycle input in the update kernel
    float* y32() const {
        return (amg(c) && mixed(c) && c->o.precision != MSP_MIXED_BF16) ? static_cast<float*>(w->vy[0]) : nullptr;
    }
    Bf16* y16() const {
        return (amg(c) && c->o.precision == MSP_MIXED_BF16) ? static_cast<Bf16*>(w->vy[0]) : nullptr;
    }

    // <r,r>, U^T r and the convergence check (initial: the active flags)
    void update_dots(bool upd) {
        Work& W = *w;
        const double wu = ubytes();
        const double bytes = (upd ? 3.0 : 1.0) * vb() + (kl ? nb * S * kl * wu : 0.0) + (y32() ? 4.0 * nb * C : 0.0) +
                             (y16() ? 2.0 * nb * C : 0.0);
        timed(c, KD_UPDATE, bytes, st, [&] {
            if (c->U16)
                HIPCHECK(launch_update_dots<Bf16>(st, C, nbu, upd, kl, nb, W.r, W.q, alpha,
                                                  static_cast<const Bf16*>(c->d_U), S, m, W.pp1, W.plrc, y32(),
                                                  y16(), c->gate));
            else if (c->U32 || !c->d_U)
                HIPCHECK(launch_update_dots<float>(st, C, nbu, upd, kl, nb, W.r, W.q, alpha,
                                                   static_cast<const float*>(c->d_U), S, m, W.pp1, W.plrc, y32(),
                                                   y16(), c->gate));
            else
                HIPCHECK(launch_update_dots<double>(st, C, nbu, upd, kl, nb, W.r, W.q, alpha,
                                                    static_cast<const double*>(c->d_U), S, m, W.pp1, W.plrc, y32(),
                                                    y16(), c->gate));
        }, [&] {
            const char* tu = c->U16 ? "Bf16" : ((c->U32 || !c->d_U) ? "float" : "double");
            return "k_update_dots<" + std::to_string(C) + ", " + (upd ? "true" : "false") + ", " +
                   std::to_string(kl > 8 ? 16 : (kl > 0 ? 8 : 0)) + ", " + tu + ">";
        });
        HIPCHECK(launch_fin_check(st, C, nbu, !upd, O, m, W.pp1, W.plrc, thr, c->d_lrc_coef, active, iters, flags,
                                  rnorm, c->d_lrc_W));
    }

    // z = M^{-1} r (+ low-rank corrections), <r,z>, beta and rho
    void precond_dot(bool init) {
        Work& W = *w;
        const float* s32 = nullptr;
        const Bf16* s16 = nullptr;
        if (amg(c) && c->o.precision == MSP_MIXED_BF16) {
            Bf16* y0 = static_cast<Bf16*>(W.vy[0]);   // written by the update kernel
            Bf16* s0 = static_cast<Bf16*>(W.vs[0]);
            vcycle<Bf16>(c, W, st, 0, y0, s0);
            s16 = s0;
        } else if (amg(c) && mixed(c)) {
            float* y0 = static_cast<float*>(W.vy[0]);   // written by the update kernel
            float* s0 = static_cast<float*>(W.vs[0]);
            vcycle<float>(c, W, st, 0, y0, s0);
            s32 = s0;
        } else {
            precondition_base(c, W, st, W.r, W.z, true);
        }
        const double wu = ubytes();
        double* z2 = init ? W.p : nullptr;   // the first search direction p = z
        const bool fq = flexible && !init;   // <q, z> for the flexible beta
        const double* qf = fq ? W.q : nullptr;
        double* pqz = fq ? W.pp2 : nullptr;
        // the mixed modes store no z (the p update rebuilds it); the first call writes p = z
        double* zs = (s16 || s32) ? nullptr : W.z;
        const double bytes = (s16 ? 2.0 : (s32 ? 4.0 : 8.0)) * nb * C + (init ? 1.0 : 0.0) * vb() +
                             (zs ? vb() : 0.0) + vb() + (fq ? vb() : 0.0) + (kl ? nb * S * kl * wu : 0.0);
        const void* U = lrc_amg ? c->d_U : nullptr;
        timed(c, KD_CAST, bytes, st, [&] {
            if (s16) {
                if (c->U16)
                    HIPCHECK((launch_zfinish<Bf16, Bf16>(st, C, nbz, nb, s16, zs, W.r, static_cast<const Bf16*>(U),
                                                         c->d_lrc_W, S, kl, m, W.pp1, z2, qf, pqz, c->gate)));
                else if (c->U32 || !c->d_U)
                    HIPCHECK((launch_zfinish<Bf16, float>(st, C, nbz, nb, s16, zs, W.r, static_cast<const float*>(U),
                                                          c->d_lrc_W, S, kl, m, W.pp1, z2, qf, pqz, c->gate)));
                else
                    HIPCHECK((launch_zfinish<Bf16, double>(st, C, nbz, nb, s16, zs, W.r,
                                                           static_cast<const double*>(U), c->d_lrc_W, S, kl, m,
                                                           W.pp1, z2, qf, pqz, c->gate)));
            } else if (s32) {
                if (c->U32 || !c->d_U)
                    HIPCHECK((launch_zfinish<float, float>(st, C, nbz, nb, s32, zs, W.r, static_cast<const float*>(U),
                                                           c->d_lrc_W, S, kl, m, W.pp1, z2, qf, pqz, c->gate)));
                else
                    HIPCHECK((launch_zfinish<float, double>(st, C, nbz, nb, s32, zs, W.r,
                                                            static_cast<const double*>(U), c->d_lrc_W, S, kl, m,
                                                            W.pp1, z2, qf, pqz, c->gate)));
            } else {
                if (c->U32 || !c->d_U)
                    HIPCHECK((launch_zfinish<double, float>(st, C, nbz, nb, W.z, W.z, W.r,
                                                            static_cast<const float*>(U), c->d_lrc_W, S, kl, m,
                                                            W.pp1, z2, qf, pqz, c->gate)));
                else
                    HIPCHECK((launch_zfinish<double, double>(st, C, nbz, nb, W.z, W.z, W.r,
                                                             static_cast<const double*>(U), c->d_lrc_W, S, kl, m,
                                                             W.pp1, z2, qf, pqz, c->gate)));
            }
        }, [&] {
            const char* ts = s16 ? "Bf16" : (s32 ? "float" : "double");
            const char* tu = c->U16 ? "Bf16" : ((c->U32 || !c->d_U) ? "float" : "double");
            return "k_zfinish<" + std::to_string(C) + ", " + ts + ", " + (U && kl > 0 ? "true" : "false") + ", " + tu +
                   ", " + (fq ? "true" : "false") + ">";
        });
        HIPCHECK(launch_fin_beta(st, C, nbz, init, flexible, W.pp1, W.pp2, active, pq, rho, beta, rz, c->gate));
    }

    void begin(const double* d_b) {
        Work& W = *w;
        d_b0 = d_b;
        vc_on = vcycle_timed(c);
        vc_ms0 = vcycle_ms(c);
        HIPCHECK(launch_colnorm2(st, n, m, d_b, W.pp1, std::min<int64_t>(512, (n + 255) / 256), bn2));
        HIPCHECK(launch_thresholds(st, C, S, m, c->o.tol, bn2, thr));
        if (S * m < C) HIPCHECK(launch_fill<double>(st, nb * C, W.r, 0.0));   // padded columns (Q_s writes the rest)
        HIPCHECK(launch_fill<double>(st, nb * C, W.x, 0.0));
        HIPCHECK(launch_fill<int>(st, 64 * 2 + 2, active, 0));   // active, iterations, flags (all 64 slots)
        HIPCHECK(launch_fill<double>(st, 64, alpha, 0.0));
        timed(c, KD_QS, 16.0 * n * m + 8.0 * n, st,   // bhat = Q_s b
              [&] { HIPCHECK(launch_qs_forward(st, S, nb, m, C, n, c->d_img, d_b, W.r)); },
              [&] { return "k_qs_forward<" + std::to_string(S) + ">"; });
        update_dots(false);
        precond_dot(true);   // also writes p = z
    }

    void half_a() {
        Work& W = *w;
        const double opb = spmm_bytes<double>(c->dAinn, C, false, &c->dsig, S);   // p read once, q written once
        timed(c, KD_OP, opb, st, [&] {   // q = Ahat p and <p, q>
            HIPCHECK(launch_op_dot(st, C, nbo, nb, c->dAinn.rp, c->dAinn.ci, c->dAinn.v64, op_sell_ref(), c->dsig.d, S,
                                   m, W.p, W.q, W.pp1, c->gate));
        }, [&] { return "k_op_dot<" + std::to_string(C) + ", " + (op_sliced() ? "true" : "false") + ">"; });
        HIPCHECK(launch_fin_alpha(st, C, nbo, W.pp1, active, rho, alpha, pq, flags));
        update_dots(true);
        x_pending = true;   // x += alpha p follows with the p update (or in finish)
    }

    void half_b() {
        Work& W = *w;
        precond_dot(false);
        const Bf16* sb = cycle_out16();
        const float* sf = cycle_out32();
        if (!sb && !sf) {
            timed(c, KD_PUPDATE, 5.0 * vb(), st,
                  [&] { HIPCHECK(launch_pcg_pupdate(st, C, nb, W.x, W.p, W.z, alpha, beta, active, c->gate != nullptr)); },
                  [&] { return "k_pcg_pupdate<" + std::to_string(C) + ">"; });
        } else {
            // z = s + U W rebuilt per row: s (and U) are read instead of a stored FP64 z
            const void* U = lrc_amg ? c->d_U : nullptr;
            const double bytes = 4.0 * vb() + (sb ? 2.0 : 4.0) * nb * C + (kl ? nb * S * kl * ubytes() : 0.0);
            const bool g = c->gate != nullptr;
            timed(c, KD_PUPDATE, bytes, st, [&] {
                if (sb && c->U16)
                    HIPCHECK((launch_pupdate_rebuild<Bf16, Bf16>(st, C, nbp, nb, W.x, W.p, sb, static_cast<const Bf16*>(U),
                                                                 c->d_lrc_W, S, kl, m, alpha, beta, active, g)));
                else if (sb && (c->U32 || !c->d_U))
                    HIPCHECK((launch_pupdate_rebuild<Bf16, float>(st, C, nbp, nb, W.x, W.p, sb,
                                                                  static_cast<const float*>(U), c->d_lrc_W, S, kl, m,
                                                                  alpha, beta, active, g)));
                else if (sb)
                    HIPCHECK((launch_pupdate_rebuild<Bf16, double>(st, C, nbp, nb, W.x, W.p, sb,
                                                                   static_cast<const double*>(U), c->d_lrc_W, S, kl, m,
                                                                   alpha, beta, active, g)));
                else if (c->U32 || !c->d_U)
                    HIPCHECK((launch_pupdate_rebuild<float, float>(st, C, nbp, nb, W.x, W.p, sf,
                                                                   static_cast<const float*>(U), c->d_lrc_W, S, kl, m,
                                                                   alpha, beta, active, g)));
                else
                    HIPCHECK((launch_pupdate_rebuild<float, double>(st, C, nbp, nb, W.x, W.p, sf,
                                                                    static_cast<const double*>(U), c->d_lrc_W, S, kl,
                                                                    m, alpha, beta, active, g)));
            }, [&] {
                const char* tu = c->U16 ? "Bf16" : ((c->U32 || !c->d_U) ? "float" : "double");
                return std::string("k_pupdate_rebuild<") + std::to_string(C) + ", " + (sb ? "Bf16" : "float") + ", " +
                       (U && kl > 0 ? "true" : "false") + ", " + tu + ">";
            });
        }
        x_pending = false;
    }

    // The host decides whether to iterate on: the device publishes the two flags and a
    // sequence number into fine-grained host memory and the host waits for that number
    // (polling memory wakes up sooner than a stream synchronisation).  Every 1024 polls
    // the stream is queried; once it has drained without the number showing, the
    // flags are copied the ordinary way.
    void read_flags() {
        Work& W = *w;
        const int seq = ++W.pub_seq;
        HIPCHECK(launch_publish_flags(st, flags, W.d_pub, seq));
        volatile int* hp = W.h_pub;
        bool seen = false;
        for (int64_t spin = 1; !seen; ++spin) {
            if (hp[2] == seq) {
                seen = true;
                break;
            }
            if ((spin & 1023) == 0) {
                const hipError_t q = hipStreamQuery(st);
                if (q == hipSuccess) {
                    seen = hp[2] == seq;
                    break;
                }
                if (q != hipErrorNotReady) HIPCHECK(q);
            }
        }
        if (seen) {
            std::atomic_thread_fence(std::memory_order_acquire);
            W.h_flags[0] = hp[0];
            W.h_flags[1] = hp[1];
        } else {
            HIPCHECK(hipMemcpyAsync(W.h_flags, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
        }
    }

    // Q_s backward and statistics (status: MSP_OK / MSP_NOT_CONVERGED / breakdown)
    int finish(double* d_x, int status, double seconds, msp_stats* out) {
        Work& W = *w;
        // x = Q_s xhat; when the last iteration stopped before its p update, its
        // x step is applied inside the transform (xhat + alpha p)
        const bool xp = x_pending;
        x_pending = false;
        timed(c, KD_QS, (xp ? 24.0 : 16.0) * n * m + 8.0 * n, st, [&] {
            HIPCHECK(launch_qs_backward(st, S, nb, m, C, n, c->d_img, W.x, d_x, xp ? W.p : nullptr,
                                        xp ? alpha : nullptr));
        }, [&] { return "k_qs_backward<" + std::to_string(S) + ">"; });
        const bool tr = c->o.true_residual != 0 && status != MSP_ERR_BREAKDOWN;
        if (tr) {
            // b - A x from the returned x: Q_s is orthogonal, so ||b - A x|| = ||bhat - Ahat xhat|| with
            // bhat = Q_s b and xhat = Q_s x formed afresh (r, q, p are free once x is out)
            HIPCHECK(launch_qs_forward(st, S, nb, m, C, n, c->d_img, d_b0, W.r));
            HIPCHECK(launch_qs_forward(st, S, nb, m, C, n, c->d_img, d_x, W.q));
            HIPCHECK((launch_spmm<double, double>(st, C, nb, c->dAinn.rp, c->dAinn.ci, c->dAinn.v64, W.q, W.p, W.r,
                                                  -1.0, 1.0, c->dsig.d, S, m, 1, false, nullptr)));
            dot(c, W, st, W.p, W.p, W.scal + SC_TRUE * 64);
        }
        HIPCHECK(hipMemcpyAsync(W.h_iters, iters, 64 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipMemcpyAsync(W.h_scal, W.scal, SC_COUNT * 64 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipMemcpyAsync(W.h_flags, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        resolve_timers(c);
        if (status == MSP_OK && W.h_flags[0]) status = MSP_ERR_BREAKDOWN;
        if (status == MSP_OK && W.h_flags[1] > 0) status = MSP_NOT_CONVERGED;
        msp_stats& R = c->stats;
        R.iters = 0;
        for (int q = 0; q < S * m; ++q) R.iters = std::max(R.iters, W.h_iters[q]);
        for (int j = 0; j < 64; ++j) R.relres_rec[j] = 0.0;
        for (int j = 0; j < m && j < 64; ++j) {
            double s2 = 0.0;
            for (int a = 0; a < S; ++a) {
                const double v = W.h_scal[SC_RNORM * 64 + a * m + j];
                s2 += v * v;
            }
            const double bn = std::sqrt(W.h_scal[SC_BN2 * 64 + j]);
            R.relres_rec[j] = bn > 0 ? std::sqrt(s2) / bn : 0.0;
        }
        for (int j = 0; j < 64; ++j) R.relres_true[j] = -1.0;
        if (tr)
            for (int j = 0; j < m && j < 64; ++j) {
                double s2 = 0.0;
                for (int a = 0; a < S; ++a) s2 += W.h_scal[SC_TRUE * 64 + a * m + j];
                const double bn = std::sqrt(W.h_scal[SC_BN2 * 64 + j]);
                R.relres_true[j] = bn > 0 ? std::sqrt(s2) / bn : 0.0;
            }
        R.t_vcycle_s = -1.0;
        if (vc_on) R.t_vcycle_s = (vcycle_ms(c) - vc_ms0) * 1e-3;
        R.status = status;
        R.t_solve_s = seconds;
        if (out) *out = R;
        return status;
    }
};

static int solve_device(msp_ctx* c, int m, const double* d_b, double* d_x, hipStream_t st, msp_stats* out,
                        Work* noalloc = nullptr) {
    if (!d_b || !d_x) throw Error(MSP_ERR_ARG, "need device arrays");
    if (c->values_invalid)
        throw Error(MSP_ERR_ARG, "the last re-setup failed: the values are invalid until msp_refresh succeeds");
    SolvePlan P(c, m, st, noalloc);
    struct SeqKeep {   // the published-flag sequence of the context's shared host buffers
        msp_ctx* c;
        Work* w;
        ~SeqKeep() {
            if (w) c->nopub_seq = w->pub_seq;
        }
    } keep{c, noalloc};
    const auto t0 = std::chrono::steady_clock::now();
    P.begin(d_b);
    P.read_flags();
    if (P.w->h_flags[0]) {   // before any iteration: the right-hand side itself
        P.finish(d_x, MSP_ERR_BREAKDOWN, 0.0, out);
        throw Error(MSP_ERR_BREAKDOWN, "non-finite value in the right-hand side");
    }
    int status = MSP_OK;
    int nactive = P.w->h_flags[1];
    int it = 0;
    while (status == MSP_OK && nactive > 0 && it < c->o.maxit) {
        P.half_a();
        P.read_flags();
        ++it;
        if (P.w->h_flags[0]) {
            status = MSP_ERR_BREAKDOWN;
            break;
        }
        nactive = P.w->h_flags[1];
        if (nactive == 0) break;
        P.half_b();
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    status = P.finish(d_x, status, secs, out);
    if (status == MSP_ERR_BREAKDOWN) throw Error(MSP_ERR_BREAKDOWN, "PCG breakdown: p^T A p <= 0 or not finite");
    return status;
}

static void fill_stats(msp_ctx* c) {
    msp_stats& st = c->stats;
    const auto& L = c->hier.lev;
    st.nlev = static_cast<int32_t>(L.size());
    double tot = 0.0;
    for (size_t l = 0; l < L.size() && l < 32; ++l) {
        st.rows[l] = L[l].A.nr;
        st.nnz[l] = L[l].A.nnz();
        tot += static_cast<double>(L[l].A.nnz());
    }
    const double nnz0 = L.empty() ? 1.0 : static_cast<double>(std::max<int64_t>(1, L[0].A.nnz()));
    st.op_complexity = tot / nnz0;
    if (L.size() > 1) {
        st.c_rat = static_cast<double>(L[1].A.nr) / static_cast<double>(L[0].A.nr);
        st.avg_nnzr = static_cast<double>(L[1].A.nnz()) / static_cast<double>(std::max<int64_t>(1, L[1].A.nr));
    } else {
        st.c_rat = 1.0;
        st.avg_nnzr = L.empty() ? 0.0 : static_cast<double>(L[0].A.nnz()) / static_cast<double>(L[0].A.nr);
    }
}

void build_lrc(msp_ctx* c);   // low-rank corrections (below)
void build_schur_lrc(msp_ctx* c);
void refresh_device(msp_ctx* c, const double* d_val, hipStream_t st);   // numeric re-setup (below)
void fv_kappa_grad(msp_fv* f, const double* d_kap, int m, const double* d_lam, const double* d_p, double* d_grad,
                   hipStream_t st);   // fv.cpp
void fv_assemble_device(msp_fv* f, const double* d_kap, double* d_val, hipStream_t st);   // fv.cpp

}  // namespace msp

// ====================================================================== C ABI

using msp::Error;

template <typename F>
static int guarded(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        msp::g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        msp::g_last_error = "host allocation failed";
        return MSP_ERR_OOM;
    } catch (const std::exception& e) {
        msp::g_last_error = e.what();
        return MSP_ERR_ARG;
    } catch (...) {
        msp::g_last_error = "unknown error";
        return MSP_ERR_ARG;
    }
}

static void check_opts(const msp_opts* o) {
    if (!o) throw Error(MSP_ERR_ARG, "null options");
    if (o->precision < MSP_FP64 || o->precision > MSP_MIXED_BF16) throw Error(MSP_ERR_ARG, "precision");
    if (o->pc < MSP_PC_AMGR || o->pc > MSP_PC_AMGS) throw Error(MSP_ERR_ARG, "pc");
    if (o->amgs_light != 0 && o->amgs_light != 1) throw Error(MSP_ERR_ARG, "amgs_light must be 0 or 1");
    if (!(o->schur_tau >= 0.0) || !std::isfinite(o->schur_tau)) throw Error(MSP_ERR_ARG, "schur_tau must be >= 0");
    if (o->pc == MSP_PC_AMGS && o->precision != MSP_FP64)
        throw Error(MSP_ERR_UNSUPPORTED, "AMGS runs in FP64 only");
    if (o->lrc_k < 0 || o->dist < 1 || o->jacobi0 < 1 || o->jacobi < 1 || o->coarse_max < 1 || o->max_levels < 1 ||
        !(o->theta >= 0.0) || !(o->tol > 0.0) || o->maxit < 0 || !(o->trunc0 >= 0.0 && o->trunc0 < 1.0))
        throw Error(MSP_ERR_ARG, "invalid option value");
    if (o->lrc_k > 0 && o->pc == MSP_PC_NONE) throw Error(MSP_ERR_ARG, "low-rank corrections need a preconditioner");
    if (o->lrc_k > 16) throw Error(MSP_ERR_UNSUPPORTED, "low-rank correction rank above 16");
    if (o->coarse64 != 0 && o->coarse64 != 1) throw Error(MSP_ERR_ARG, "coarse64 must be 0 or 1");
    if (o->max_levels > msp::kMaxLevels) throw Error(MSP_ERR_UNSUPPORTED, "more than 32 levels");
    if (o->nu1 < 1 || o->nu1 > 8 || o->nu2 < 1 || o->nu2 > 8) throw Error(MSP_ERR_ARG, "nu1 and nu2 must be in 1..8");
    if (o->nu1 != o->nu2)
        throw Error(MSP_ERR_UNSUPPORTED, "nu1 != nu2 makes the V-cycle non-symmetric, which PCG cannot take");
    if (o->true_residual != 0 && o->true_residual != 1) throw Error(MSP_ERR_ARG, "true_residual must be 0 or 1");
    if (o->afsai_nnz < 0 || o->afsai_nnz > 64) throw Error(MSP_ERR_ARG, "afsai_nnz must be in 0..64");
    if (o->emin_steps < 0 || o->emin_steps > 100) throw Error(MSP_ERR_ARG, "emin_steps must be in 0..100");
    if (o->pc == MSP_PC_AMGS && (o->afsai_nnz > 0 || o->emin_steps > 0))
        throw Error(MSP_ERR_UNSUPPORTED, "AMGS keeps its own FSAIs and the plain interpolation");
}

// Host part of the setup: blocks, validation, hierarchy (no HIP calls).
static std::unique_ptr<msp_ctx> setup_host(const msp_csr* A, const msp_symmap* map, const msp_opts* o) {
    std::unique_ptr<msp_ctx> c(new msp_ctx());
    c->o = *o;
    c->device = o->device;
    c->lrc_k = o->lrc_k;
    c->sym = msp::extract_blocks(A, map);
    if (o->pc == MSP_PC_AMGS) {
        c->am = msp::build_amgs(c->sym, *o);   // reorders the base cells inner first
        c->hier = std::move(c->am.HK);
        c->am.HK = msp::HostHierarchy{};
    } else if (o->pc == MSP_PC_AMGR || o->pc == MSP_PC_AMGR_SUB) {
        c->hier = msp::build_hierarchy(c->sym.Ainn, c->sym.iface, *o);
        if (o->pc == MSP_PC_AMGR_SUB && c->hier.lev.size() > 1) {
            c->subv = msp::build_sub_values(c->hier, c->sym.sigma, c->sym.iface, 1 << c->sym.s, *o);
            c->sub = true;
        }
    } else {
        c->hier.lev.emplace_back();
        c->hier.lev.back().A = c->sym.Ainn;
        if (o->pc == MSP_PC_FSAI) c->Gf = msp::fsai_full_lower(c->sym.Ainn);
    }
    msp::fill_stats(c.get());
    c->stats.split_drift = -1;
    c->stats.split_drift1 = -1;
    return c;
}

// Host part of the setup for a domain made of copies: one subsystem holding the
// whole matrix, level 0 split by the replicated populated interface.
static std::unique_ptr<msp_ctx> setup_host_copies(const msp_csr* A, const msp_copies* map, const msp_opts* o) {
    if (o->pc == MSP_PC_AMGR_SUB || o->pc == MSP_PC_AMGS)
        throw Error(MSP_ERR_ARG, "a domain of copies is solved in its own basis: use MSP_PC_AMGR");
    std::unique_ptr<msp_ctx> c(new msp_ctx());
    c->o = *o;
    c->device = o->device;
    c->lrc_k = o->lrc_k;
    msp::CopyParts parts = msp::extract_copies(A, map, *o);
    c->sym = std::move(parts.sym);
    c->copies = true;
    if (o->pc == MSP_PC_AMGR) {
        c->hier = msp::build_hierarchy(c->sym.Ainn, c->sym.iface, *o, &parts.cf0);
    } else {
        c->hier.lev.emplace_back();
        c->hier.lev.back().A = c->sym.Ainn;
        if (o->pc == MSP_PC_FSAI) c->Gf = msp::fsai_full_lower(c->sym.Ainn);
    }
    msp::fill_stats(c.get());
    c->stats.split_drift = -1;
    c->stats.split_drift1 = -1;
    return c;
}

// Host part of a rebuild below the reduction level: the blocks and the reduction
// level of `old` with its current values (after a device re-setup: fetched), every
// level below built afresh from its level-1 operator; the per-subsystem values too,
// or (sub_later) the shared ones in their place, for a device re-setup to replace.
static std::unique_ptr<msp_ctx> setup_host_below(msp_ctx* old, bool sub_later) {
    if (old->values_invalid) throw Error(MSP_ERR_ARG, "the context's values are invalid (a re-setup failed)");
    if (old->o.pc != MSP_PC_AMGR && old->o.pc != MSP_PC_AMGR_SUB)
        throw Error(MSP_ERR_UNSUPPORTED, "a rebuild below the reduction level needs an AMGR context");
    if (old->hier.lev.size() < 2) throw Error(MSP_ERR_ARG, "the hierarchy has no level below the reduction level");
    if (old->on_device) msp::sync_host(old);
    std::unique_ptr<msp_ctx> c(new msp_ctx());
    c->o = old->o;
    c->device = old->device;
    c->lrc_k = old->lrc_k;
    c->sym = old->sym;
    c->copies = old->copies;
    c->hier = msp::build_hierarchy_below(old->hier, c->o);
    if (old->sub) {
        c->subv = sub_later ? msp::replicated_sub_values(c->hier, 1 << c->sym.s)
                            : msp::build_sub_values(c->hier, c->sym.sigma, c->sym.iface, 1 << c->sym.s, c->o);
        c->sub = true;
    }
    msp::fill_stats(c.get());
    c->stats.split_drift = -1;
    c->stats.split_drift1 = -1;
    return c;
}

// Device part: upload and low-rank corrections.
static void setup_device(msp_ctx* c) {
    int ndev = 0;
    HIPCHECK(hipGetDeviceCount(&ndev));
    if (c->o.device >= ndev) throw Error(MSP_ERR_ARG, "device ordinal out of range");
    msp::upload_all(c);
    HIPCHECK(msp::scratch_init());   // the allocation-free solve's workspace on this device
    msp::alloc_host_bufs(c->nohb);
    if (c->lrc_k > 0 && c->o.pc == MSP_PC_AMGS) msp::build_schur_lrc(c);
    else if (c->lrc_k > 0) msp::build_lrc(c);
    HIPCHECK(hipDeviceSynchronize());
}

// ====================================================================== batched solves

struct msp_batch {
    std::vector<msp_ctx*> sys;
    std::vector<hipStream_t> streams;
    hipStream_t main = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    // graph of `cap` gated iterations of every system (the whole solve in one launch), cached for one
    // vector of m and one cap; a one-iteration graph continues a solve that needs more
    std::vector<int> graph_m;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph1 = nullptr;
    hipGraphExec_t exec1 = nullptr;
    int cap = 16;          // iterations the next solve's graph holds
    int cap_built = 0;     // iterations the cached graph holds
    int launches = 0;      // graph launches of the last solve
    int** d_flag_ptrs = nullptr;
    int* d_flags = nullptr;
    int* h_flags = nullptr;
    ~msp_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (exec1) (void)hipGraphExecDestroy(exec1);
        if (graph1) (void)hipGraphDestroy(graph1);
        for (auto e : joins) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        for (auto s : streams) (void)hipStreamDestroy(s);
        if (main) (void)hipStreamDestroy(main);
        if (d_flag_ptrs) (void)hipFree(d_flag_ptrs);
        if (d_flags) (void)hipFree(d_flags);
        if (h_flags) (void)hipHostFree(h_flags);
        for (auto c : sys) delete c;
    }
};

namespace msp {

static void batch_setup(int nsys, const msp_csr* A, const msp_symmap* maps, const msp_opts* o, msp_batch** out) {
    if (nsys <= 0 || !A || !maps || !out) throw Error(MSP_ERR_ARG, "bad batch arguments");
    check_opts(o);
    if (o->device < 0) throw Error(MSP_ERR_ARG, "batched solves need a device");
    if (o->pc == MSP_PC_AMGS) throw Error(MSP_ERR_UNSUPPORTED, "batched solves with AMGS");
    std::unique_ptr<msp_batch> bt(new msp_batch());
    bt->sys.assign(nsys, nullptr);
    // host setups in parallel (each context is independent)
    std::vector<std::unique_ptr<msp_ctx>> hosts(nsys);
    std::vector<std::string> errs(nsys);
    std::vector<int> codes(nsys, MSP_OK);
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::atomic<int> next(0);
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nth; ++t)
        pool.emplace_back([&]() {
            for (int i = next++; i < nsys; i = next++) {
                try {
                    hosts[i] = setup_host(&A[i], &maps[i], o);
                } catch (const Error& e) {
                    codes[i] = e.status;
                    errs[i] = e.what();
                } catch (const std::exception& e) {
                    codes[i] = MSP_ERR_ARG;
                    errs[i] = e.what();
                }
            }
        });
    for (auto& th : pool) th.join();
    for (int i = 0; i < nsys; ++i)
        if (codes[i] != MSP_OK) throw Error(codes[i], "system " + std::to_string(i) + ": " + errs[i]);
    HIPCHECK(hipSetDevice(o->device));
    for (int i = 0; i < nsys; ++i) {
        setup_device(hosts[i].get());
        bt->sys[i] = hosts[i].release();
    }
    bt->streams.resize(nsys);
    bt->joins.resize(nsys);
    for (int i = 0; i < nsys; ++i) {
        HIPCHECK(hipStreamCreateWithFlags(&bt->streams[i], hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&bt->joins[i], hipEventDisableTiming));
    }
    HIPCHECK(hipStreamCreateWithFlags(&bt->main, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&bt->fork, hipEventDisableTiming));
    HIPCHECK(hipMalloc(&bt->d_flag_ptrs, sizeof(int*) * nsys));
    HIPCHECK(hipMalloc(&bt->d_flags, sizeof(int) * 2 * nsys));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void**>(&bt->h_flags), sizeof(int) * 2 * nsys, hipHostMallocDefault));
    *out = bt.release();
}

// Solve every system: an eager start per system on its own stream, then one
// launch of a captured graph holding `cap` iterations of every system on
// parallel branches.  The iterations are gated on the device: every kernel
// of a system whose columns have all converged returns at once (its p update
// stops once every step is zero), so each system does the iterations it
// needs and the host reads the flags once.  A system still active after the
// graph continues by one-iteration graph launches up to maxit.  The next
// solve's graph holds the iterations this one needed (at most maxit): a
// gated kernel returns at once but still dispatches its grid, so extra
// iterations are not free.  The graph is captured again when a solve needs
// more iterations than it holds or leaves two or more of them unused, or
// when the vector of m changes.
static int batch_solve(msp_batch* bt, const int32_t* m, const double* const* d_b, double* const* d_x,
                       hipStream_t user, msp_stats* st) {
    const int nsys = static_cast<int>(bt->sys.size());
    if (!m || !d_b || !d_x) throw Error(MSP_ERR_ARG, "null batch arrays");
    HIPCHECK(hipSetDevice(bt->sys[0]->device));
    std::vector<std::unique_ptr<SolvePlan>> plans(nsys);
    for (int i = 0; i < nsys; ++i) {
        if (!d_b[i] || !d_x[i]) throw Error(MSP_ERR_ARG, "null device array in batch");
        std::fill(bt->sys[i]->tm.on.begin(), bt->sys[i]->tm.on.end(), 0);
        plans[i].reset(new SolvePlan(bt->sys[i], m[i], bt->streams[i]));
    }
    int maxit = 0;
    for (auto c : bt->sys) maxit = std::max(maxit, c->o.maxit);
    const int cap = std::max(1, std::min(bt->cap, maxit));
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHECK(hipEventRecord(bt->fork, user));
    for (int i = 0; i < nsys; ++i) {
        HIPCHECK(hipStreamWaitEvent(bt->streams[i], bt->fork, 0));
        plans[i]->begin(d_b[i]);
    }
    // device pointers of every system's flags
    std::vector<int*> ptrs(nsys);
    for (int i = 0; i < nsys; ++i) ptrs[i] = plans[i]->flags;
    HIPCHECK(hipMemcpy(bt->d_flag_ptrs, ptrs.data(), sizeof(int*) * nsys, hipMemcpyHostToDevice));
    for (int i = 0; i < nsys; ++i) HIPCHECK(hipStreamSynchronize(bt->streams[i]));
    std::vector<int> mv(m, m + nsys);
    // graph of `iters` gated iterations of every system on parallel branches, then the flags gathered
    auto capture = [&](int iters, hipGraph_t* g, hipGraphExec_t* ex) {
        if (*ex) (void)hipGraphExecDestroy(*ex);
        if (*g) (void)hipGraphDestroy(*g);
        *ex = nullptr;
        *g = nullptr;
        for (int i = 0; i < nsys; ++i) bt->sys[i]->gate = plans[i]->active;
        try {
            HIPCHECK(hipStreamBeginCapture(bt->main, hipStreamCaptureModeRelaxed));
            HIPCHECK(hipEventRecord(bt->fork, bt->main));
            for (int i = 0; i < nsys; ++i) {
                HIPCHECK(hipStreamWaitEvent(bt->streams[i], bt->fork, 0));
                for (int k = 0; k < iters; ++k) {
                    plans[i]->half_a();
                    plans[i]->half_b();
                }
                HIPCHECK(hipEventRecord(bt->joins[i], bt->streams[i]));
                HIPCHECK(hipStreamWaitEvent(bt->main, bt->joins[i], 0));
            }
            HIPCHECK(launch_gather_flags(bt->main, nsys, bt->d_flag_ptrs, bt->d_flags));
            HIPCHECK(hipStreamEndCapture(bt->main, g));
        } catch (...) {
            for (auto c : bt->sys) c->gate = nullptr;
            throw;
        }
        for (auto c : bt->sys) c->gate = nullptr;
        HIPCHECK(hipGraphInstantiate(ex, *g, nullptr, nullptr, 0));
    };
    if (!bt->exec || mv != bt->graph_m || bt->cap_built != cap) {
        capture(cap, &bt->graph, &bt->exec);
        capture(1, &bt->graph1, &bt->exec1);
        bt->graph_m = mv;
        bt->cap_built = cap;
    }
    auto read_flags = [&] {
        HIPCHECK(hipMemcpyAsync(bt->h_flags, bt->d_flags, sizeof(int) * 2 * nsys, hipMemcpyDeviceToHost, bt->main));
        HIPCHECK(hipStreamSynchronize(bt->main));
        bool any = false, broke = false;
        for (int i = 0; i < nsys; ++i) {
            any |= bt->h_flags[2 * i + 1] > 0;
            broke |= bt->h_flags[2 * i] != 0;
        }
        return any && !broke;
    };
    HIPCHECK(launch_gather_flags(bt->main, nsys, bt->d_flag_ptrs, bt->d_flags));
    int it = 0;
    bt->launches = 0;
    if (read_flags()) {
        HIPCHECK(hipGraphLaunch(bt->exec, bt->main));
        bt->launches = 1;
        it = cap;
        while (read_flags() && it < maxit) {
            HIPCHECK(hipGraphLaunch(bt->exec1, bt->main));
            ++bt->launches;
            ++it;
        }
    }
    HIPCHECK(hipEventRecord(bt->fork, bt->main));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = MSP_OK;
    int most = 0;
    for (int i = 0; i < nsys; ++i) {
        HIPCHECK(hipStreamWaitEvent(bt->streams[i], bt->fork, 0));
        msp_stats si{};
        const int rc = plans[i]->finish(d_x[i], MSP_OK, secs, &si);
        if (st) st[i] = si;
        most = std::max(most, si.iters);
        if (rc < worst || (worst == MSP_OK && rc != MSP_OK)) worst = rc;
    }
    for (int i = 0; i < nsys; ++i) {
        HIPCHECK(hipEventRecord(bt->joins[i], bt->streams[i]));
        HIPCHECK(hipStreamWaitEvent(user, bt->joins[i], 0));
    }
    // the next graph: this solve's count when it needed more, or when the cached graph wastes two or more
    // iterations (a gated kernel still dispatches its grid); otherwise keep the cached graph
    const int need = std::max(1, std::min(maxit, most));
    bt->cap = (need > bt->cap_built || need + 1 < bt->cap_built) ? need : bt->cap_built;
    if (worst == MSP_ERR_BREAKDOWN) throw Error(MSP_ERR_BREAKDOWN, "PCG breakdown in a batched system");
    return worst;
}

}  // namespace msp

extern "C" {

int msp_setup(const msp_csr* A, const msp_symmap* map, const msp_opts* o, msp_ctx** out) {
    return guarded([&]() -> int {
        if (!out) throw Error(MSP_ERR_ARG, "null output");
        *out = nullptr;
        check_opts(o);
        const auto t0 = std::chrono::steady_clock::now();
        std::unique_ptr<msp_ctx> c = setup_host(A, map, o);
        if (o->device >= 0) setup_device(c.get());
        const auto t1 = std::chrono::steady_clock::now();
        c->stats.t_setup_s = std::chrono::duration<double>(t1 - t0).count();
        *out = c.release();
        return MSP_OK;
    });
}

int msp_rebuild_below(msp_ctx* c, const double* d_val, void* hip_stream, msp_ctx** out) {
    return guarded([&]() -> int {
        if (!out) throw Error(MSP_ERR_ARG, "null output");
        *out = nullptr;
        if (!c) throw Error(MSP_ERR_ARG, "null context");
        if (d_val && !c->on_device) throw Error(MSP_ERR_ARG, "device values for a context without a device");
        if (d_val && c->o.precision == MSP_MIXED_FP32_BF16G)
            throw Error(MSP_ERR_UNSUPPORTED, "the re-setup of the BF16-G variant");
        const auto t0 = std::chrono::steady_clock::now();
        std::unique_ptr<msp_ctx> n = setup_host_below(c, d_val != nullptr);
        if (n->o.device >= 0 && d_val) {
            // upload without corrections; the device re-setup then computes every value
            // (per-subsystem ones included) and the corrections from the caller's matrix
            const int k = n->lrc_k;
            n->lrc_k = 0;
            setup_device(n.get());
            n->lrc_k = k;
            msp::refresh_device(n.get(), d_val, static_cast<hipStream_t>(hip_stream));
            msp::fill_stats(n.get());
        } else if (n->o.device >= 0) {
            setup_device(n.get());
        }
        const auto t1 = std::chrono::steady_clock::now();
        n->stats.t_setup_s = std::chrono::duration<double>(t1 - t0).count();
        *out = n.release();
        return MSP_OK;
    });
}

int msp_setup_copies(const msp_csr* A, const msp_copies* map, const msp_opts* o, msp_ctx** out) {
    return guarded([&]() -> int {
        if (!out) throw Error(MSP_ERR_ARG, "null output");
        *out = nullptr;
        check_opts(o);
        const auto t0 = std::chrono::steady_clock::now();
        std::unique_ptr<msp_ctx> c = setup_host_copies(A, map, o);
        if (o->device >= 0) setup_device(c.get());
        const auto t1 = std::chrono::steady_clock::now();
        c->stats.t_setup_s = std::chrono::duration<double>(t1 - t0).count();
        *out = c.release();
        return MSP_OK;
    });
}

int msp_refresh(msp_ctx* c, const double* d_val, void* hip_stream) {
    return guarded([&]() -> int {
        if (!c) throw Error(MSP_ERR_ARG, "null context");
        msp::refresh_device(c, d_val, static_cast<hipStream_t>(hip_stream));
        msp::fill_stats(c);
        return MSP_OK;
    });
}

int msp_solve_device(msp_ctx* c, int32_t m, const double* d_b, double* d_x, void* hip_stream, msp_stats* st) {
    return guarded([&]() -> int {
        if (!c) throw Error(MSP_ERR_ARG, "null context");
        return msp::solve_device(c, m, d_b, d_x, static_cast<hipStream_t>(hip_stream), st);
    });
}

int msp_solve_device_noalloc(msp_ctx* c, int32_t m, const double* d_b, double* d_x, void* hip_stream,
                             msp_stats* st) {
    return guarded([&]() -> int {
        if (!c) throw Error(MSP_ERR_ARG, "null context");
        for (char on : c->tm.on)
            if (on) throw Error(MSP_ERR_ARG, "per-kernel timers must be off for the allocation-free solve");
        msp::Work w;
        return msp::solve_device(c, m, d_b, d_x, static_cast<hipStream_t>(hip_stream), st, &w);
    });
}

int msp_solve(msp_ctx* c, int32_t m, const double* b, double* x, msp_stats* st) {
    return guarded([&]() -> int {
        if (!c || !b || !x || m <= 0) throw Error(MSP_ERR_ARG, "null argument or m <= 0");
        if (!c->on_device) throw Error(MSP_ERR_ARG, "context was set up without a device");
        HIPCHECK(hipSetDevice(c->device));
        const size_t bytes = sizeof(double) * static_cast<size_t>(c->sym.n) * static_cast<size_t>(m);
        double *db = nullptr, *dx = nullptr;
        HIPCHECK(hipMalloc(&db, bytes));
        if (hipMalloc(&dx, bytes) != hipSuccess) {
            (void)hipFree(db);
            throw Error(MSP_ERR_OOM, "device allocation failed");
        }
        int rc;
        try {
            HIPCHECK(hipMemcpy(db, b, bytes, hipMemcpyHostToDevice));
            rc = msp::solve_device(c, m, db, dx, nullptr, st);
            HIPCHECK(hipMemcpy(x, dx, bytes, hipMemcpyDeviceToHost));
        } catch (...) {
            (void)hipFree(db);
            (void)hipFree(dx);
            throw;
        }
        (void)hipFree(db);
        (void)hipFree(dx);
        return rc;
    });
}

int msp_get_stats(const msp_ctx* c, msp_stats* st) {
    if (!c || !st) return MSP_ERR_ARG;
    *st = c->stats;
    return MSP_OK;
}

int msp_num_levels(const msp_ctx* c, int32_t* nlev) {
    if (!c || !nlev) return MSP_ERR_ARG;
    *nlev = static_cast<int32_t>(c->hier.lev.size());
    return MSP_OK;
}

int msp_level_sizes(const msp_ctx* c, int32_t lev, int64_t* n, int64_t* nnz_A, int64_t* nnz_P, int64_t* nnz_G) {
    if (!c || lev < 0 || lev >= static_cast<int32_t>(c->hier.lev.size())) return MSP_ERR_ARG;
    const auto& L = c->hier.lev[lev];
    if (n) *n = L.A.nr;
    if (nnz_A) *nnz_A = L.A.nnz();
    if (nnz_P) *nnz_P = L.P.nnz();
    if (nnz_G) *nnz_G = L.G.nnz();
    return MSP_OK;
}

static void copy_csr(const msp::Csr& M, int64_t* rp, int32_t* ci, double* v) {
    if (rp && !M.rp.empty()) std::copy(M.rp.begin(), M.rp.end(), rp);
    if (ci) std::copy(M.ci.begin(), M.ci.end(), ci);
    if (v) std::copy(M.v.begin(), M.v.end(), v);
}

// The host copy of the values is a cache of the device's after a re-setup:
// exports fetch it first (blocking).
static int synced(const msp_ctx* c) {
    return guarded([&]() -> int {
        msp::sync_host(const_cast<msp_ctx*>(c));
        return MSP_OK;
    });
}

int msp_export_level(const msp_ctx* c, int32_t lev, int8_t* cf, int64_t* A_rp, int32_t* A_ci, double* A_v,
                     int64_t* P_rp, int32_t* P_ci, double* P_v, int64_t* G_rp, int32_t* G_ci, double* G_v,
                     double* omega) {
    if (!c || lev < 0 || lev >= static_cast<int32_t>(c->hier.lev.size())) return MSP_ERR_ARG;
    if (const int rc = synced(c)) return rc;
    const auto& L = c->hier.lev[lev];
    if (cf) std::copy(L.cf.begin(), L.cf.end(), cf);
    copy_csr(L.A, A_rp, A_ci, A_v);
    copy_csr(L.P, P_rp, P_ci, P_v);
    copy_csr(L.G, G_rp, G_ci, G_v);
    if (omega) *omega = L.omega;
    return MSP_OK;
}

int msp_export_sub_level(const msp_ctx* c, int32_t lev, int32_t a, double* A_v, double* P_v, double* G_v,
                         double* omega) {
    if (!c || !c->sub || lev < 1 || lev >= static_cast<int32_t>(c->hier.lev.size()) || a < 0 || a >= c->subv.S)
        return MSP_ERR_ARG;
    if (const int rc = synced(c)) return rc;
    const int S = c->subv.S;
    auto take = [&](const std::vector<double>& v, double* out) {
        if (!out) return;
        const size_t n = v.size() / S;
        for (size_t k = 0; k < n; ++k) out[k] = v[k * S + a];
    };
    take(c->subv.A[lev], A_v);
    take(c->subv.P[lev], P_v);
    take(c->subv.G[lev], G_v);
    if (omega) *omega = c->subv.omega[lev][a];
    return MSP_OK;
}

int msp_export_amgs(const msp_ctx* c, int32_t which, int64_t* nrows, int64_t* ncols, int64_t* nnz, int64_t* rp,
                    int32_t* ci, double* v) {
    return guarded([&]() -> int {
        if (!c || c->o.pc != MSP_PC_AMGS) throw Error(MSP_ERR_ARG, "not an AMGS context");
        const msp::Csr* M = nullptr;
        switch (which) {
            case 0: M = &c->am.B; break;
            case 1: M = &c->am.C1; break;
            case 2: M = &c->am.GK; break;
            case 3: M = &c->am.SG1; break;
            case 4: M = &c->am.GS1; break;
            default: throw Error(MSP_ERR_ARG, "which must be 0..4");
        }
        if (nrows) *nrows = M->nr;
        if (ncols) *ncols = M->nc;
        if (nnz) *nnz = M->nnz();
        if (rp) std::copy(M->rp.begin(), M->rp.end(), rp);
        if (ci) std::copy(M->ci.begin(), M->ci.end(), ci);
        if (v) std::copy(M->v.begin(), M->v.end(), v);
        return MSP_OK;
    });
}

int msp_export_outer(const msp_ctx* c, double* sigma, int8_t* iface) {
    if (!c) return MSP_ERR_ARG;
    if (const int rc = synced(c)) return rc;
    if (sigma) std::copy(c->sym.sigma.begin(), c->sym.sigma.end(), sigma);
    if (iface) std::copy(c->sym.iface.begin(), c->sym.iface.end(), iface);
    return MSP_OK;
}

int msp_export_lrc(const msp_ctx* c, int32_t* kept, double* ritz) {
    if (!c) return MSP_ERR_ARG;
    if (kept) std::copy(c->lrc_kept.begin(), c->lrc_kept.end(), kept);
    if (ritz) std::copy(c->lrc_ritz.begin(), c->lrc_ritz.end(), ritz);
    return MSP_OK;
}

int msp_batch_setup(int32_t nsys, const msp_csr* A, const msp_symmap* maps, const msp_opts* o, msp_batch** out) {
    return guarded([&]() -> int {
        if (out) *out = nullptr;
        msp::batch_setup(nsys, A, maps, o, out);
        return MSP_OK;
    });
}

int msp_batch_solve(msp_batch* bt, const int32_t* m, const double* const* d_b, double* const* d_x, void* hip_stream,
                    msp_stats* st) {
    return guarded([&]() -> int {
        if (!bt) throw Error(MSP_ERR_ARG, "null batch");
        return msp::batch_solve(bt, m, d_b, d_x, static_cast<hipStream_t>(hip_stream), st);
    });
}

int msp_batch_size(const msp_batch* bt, int32_t* nsys) {
    if (!bt || !nsys) return MSP_ERR_ARG;
    *nsys = static_cast<int32_t>(bt->sys.size());
    return MSP_OK;
}

int msp_batch_set_chunk(msp_batch* bt, int32_t iterations) {
    if (!bt || iterations < 1 || iterations > 1000) return MSP_ERR_ARG;
    bt->cap = iterations;
    return MSP_OK;
}

int msp_batch_last_launches(const msp_batch* bt, int32_t* launches) {
    if (!bt || !launches) return MSP_ERR_ARG;
    *launches = bt->launches;
    return MSP_OK;
}

void msp_batch_free(msp_batch* bt) { delete bt; }

int msp_set_timing(msp_ctx* c, int32_t kind, int32_t on) {
    if (!c || kind < -1 || kind >= msp::KD_COUNT) return MSP_ERR_ARG;
    if (kind == -1) std::fill(c->tm.on.begin(), c->tm.on.end(), static_cast<char>(on ? 1 : 0));
    else c->tm.on[kind] = on ? 1 : 0;
    return MSP_OK;
}

int msp_reset_timing(msp_ctx* c) {
    if (!c) return MSP_ERR_ARG;
    std::fill(c->tm.count.begin(), c->tm.count.end(), 0);
    std::fill(c->tm.ms.begin(), c->tm.ms.end(), 0.0);
    std::fill(c->tm.bytes.begin(), c->tm.bytes.end(), 0.0);
    return MSP_OK;
}

int msp_get_timing_kernel(const msp_ctx* c, int32_t kind, char* name, int32_t len) {
    if (!c || kind < 0 || kind >= msp::KD_COUNT || !name || len <= 0) return MSP_ERR_ARG;
    const std::string& v = c->tm.variant[kind];
    const size_t k = std::min(v.size(), static_cast<size_t>(len - 1));
    std::memcpy(name, v.data(), k);
    name[k] = 0;
    return MSP_OK;
}

int msp_get_timing(const msp_ctx* c, int32_t kind, int64_t* count, double* total_ms, double* total_bytes) {
    if (!c || kind < 0 || kind >= msp::KD_COUNT) return MSP_ERR_ARG;
    if (count) *count = c->tm.count[kind];
    if (total_ms) *total_ms = c->tm.ms[kind];
    if (total_bytes) *total_bytes = c->tm.bytes[kind];
    return MSP_OK;
}

int msp_fv_create(const msp_faces* F, const msp_symmap* map, int32_t device, msp_fv** out) {
    return guarded([&]() -> int {
        if (!out) throw Error(MSP_ERR_ARG, "null output");
        *out = nullptr;
        msp::fv_create(F, map, device, out);
        return MSP_OK;
    });
}

int msp_fv_nnz(const msp_fv* f, int64_t* nnz) {
    if (!f || !nnz) return MSP_ERR_ARG;
    *nnz = msp::fv_nnz(f);
    return MSP_OK;
}

int msp_fv_assemble(const msp_fv* f, const double* kappa_base, int64_t* rowptr, int32_t* col, double* val) {
    return guarded([&]() -> int {
        if (!f) throw Error(MSP_ERR_ARG, "null operator");
        msp::fv_assemble(f, kappa_base, rowptr, col, val);
        return MSP_OK;
    });
}

int msp_fv_assemble_device(msp_fv* f, const double* d_kappa_base, double* d_val, void* hip_stream) {
    return guarded([&]() -> int {
        if (!f) throw Error(MSP_ERR_ARG, "null operator");
        msp::fv_assemble_device(f, d_kappa_base, d_val, static_cast<hipStream_t>(hip_stream));
        return MSP_OK;
    });
}

int msp_fv_kappa_grad(msp_fv* f, const double* d_kappa_base, int32_t m, const double* d_lambda, const double* d_p,
                      double* d_grad, void* hip_stream) {
    return guarded([&]() -> int {
        if (!f) throw Error(MSP_ERR_ARG, "null operator");
        msp::fv_kappa_grad(f, d_kappa_base, m, d_lambda, d_p, d_grad, static_cast<hipStream_t>(hip_stream));
        return MSP_OK;
    });
}

void msp_fv_free(msp_fv* f) { msp::fv_free(f); }

void msp_free(msp_ctx* c) { delete c; }

const char* msp_last_error(void) { return msp::g_last_error.c_str(); }

}  // extern "C"

namespace msp {

// Low-rank corrections (Sec. 2.1 eq. (2.24), Sec. 2.2 eq. (2.32)), eigenpairs by
// Lanczos with full reorthogonalisation, run for all 2^s subsystems at once as
// the columns of one multivector:
//   AMGR: operator M^{-1} A_a in the A_a inner product (M^{-1} = the shared
//         V-cycle); corrections u_t (A_a-orthonormal Ritz vectors) with
//         coefficient 1 - lam_t for the k smallest Ritz values below 1.
//   FSAI: operator G A_a G^T, Euclidean; corrections v_t with coefficient
//         1/lam_t - 1, applied between the G and G^T products.
// Start vector v_i = splitmix64(seed ^ i ^ 0x1CC)/2^64 - 1/2 (all subsystems),
// max(4k, 40) steps (at most n_b).
// Lockstep Lanczos over the 2^s subsystems on n rows (one column per
// subsystem), with full reorthogonalisation; the k smallest Ritz pairs below
// one become the corrections U (n x S*k).  amg_form: op(v, B v) = M^{-1} B v
// self-adjoint in the B inner product, coefficient 1 - lambda (LRCAMG);
// otherwise op is symmetric in the Euclidean product, coefficient 1/lambda - 1
// (LRCFSAI form).
static void lanczos_corrections(msp_ctx* c, Work& w, int64_t n, bool amg_form,
                                const std::function<void(const double*, double*)>& applyB,
                                const std::function<void(const double*, const double*, double*)>& op) {
    const int S = 1 << c->sym.s;
    const int k = c->lrc_k;
    const int K = static_cast<int>(std::min<int64_t>(std::max(4 * k, 40), n));
    const int C = w.C;
    const bool amg = amg_form;
    hipStream_t st = nullptr;
    const int64_t len = n * C;
    double* V = c->dalloc<double>(static_cast<int64_t>(K) * len);
    double* BV = amg ? c->dalloc<double>(static_cast<int64_t>(K) * len) : V;
    double* hcoef = c->dalloc<double>(static_cast<int64_t>(K) * 64);
    double* dvec = c->dalloc<double>(64);
    double* wv = w.x;    // w
    double* bw = w.q;    // B w
    std::vector<double> h(64), hv(len);

    auto coldots = [&](const double* X, const double* Y, double* out_host) {
        dot(c, w, st, X, Y, dvec, n);
        HIPCHECK(hipMemcpyAsync(out_host, dvec, C * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
    };
    auto scale_into = [&](double* dst, const double* src, const std::vector<double>& f) {
        HIPCHECK(hipMemcpyAsync(dvec, f.data(), C * sizeof(double), hipMemcpyHostToDevice, st));
        if (dst != src) HIPCHECK(hipMemcpyAsync(dst, src, len * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHECK(launch_scale_cols<double>(st, len, C, dst, dvec));
    };

    // start vector, replicated over the subsystem columns (padded columns zero)
    for (int64_t i = 0; i < n; ++i) {
        const double v = unit_centered(c->o.seed ^ static_cast<uint64_t>(i) ^ 0x1CCull);
        for (int a = 0; a < C; ++a) hv[i * C + a] = a < S ? v : 0.0;
    }
    HIPCHECK(hipMemcpy(V, hv.data(), len * sizeof(double), hipMemcpyHostToDevice));
    if (amg) applyB(V, BV);
    coldots(V, BV, h.data());
    std::vector<double> f(C, 0.0);
    for (int a = 0; a < S; ++a) f[a] = 1.0 / std::sqrt(h[a]);
    scale_into(V, V, f);
    if (amg) scale_into(BV, BV, f);

    std::vector<std::vector<double>> alpha(S), beta(S);
    std::vector<int> nsteps(S, 0);
    std::vector<char> live(S, 1);
    std::vector<double> al(64), b2(64);
    for (int j = 0; j < K; ++j) {
        double* Vj = V + static_cast<int64_t>(j) * len;
        double* BVj = BV + static_cast<int64_t>(j) * len;
        op(Vj, BVj, wv);
        coldots(wv, BVj, al.data());
        // classical Gram-Schmidt, twice, against every basis vector so far
        for (int pass = 0; pass < 2; ++pass) {
            for (int i = 0; i <= j; ++i)
                dot(c, w, st, wv, BV + static_cast<int64_t>(i) * len, hcoef + static_cast<int64_t>(i) * 64, n);
            for (int i = 0; i <= j; ++i)
                HIPCHECK(launch_axpy_cols(st, len, C, wv, V + static_cast<int64_t>(i) * len,
                                          hcoef + static_cast<int64_t>(i) * 64));
        }
        if (amg) applyB(wv, bw);
        coldots(wv, amg ? bw : wv, b2.data());
        for (int a = 0; a < S; ++a) {
            if (!live[a]) continue;
            alpha[a].push_back(al[a]);
            nsteps[a] = j + 1;
            const double b = std::sqrt(std::max(b2[a], 0.0));
            if (j == K - 1 || b <= 1e-13 * std::fabs(al[a])) {
                live[a] = 0;
                f[a] = 0.0;
            } else {
                beta[a].push_back(b);
                f[a] = 1.0 / b;
            }
        }
        if (j + 1 < K) {
            scale_into(V + static_cast<int64_t>(j + 1) * len, wv, f);
            if (amg) scale_into(BV + static_cast<int64_t>(j + 1) * len, bw, f);
        }
    }

    // Ritz pairs per subsystem: k smallest, keep those below 1
    std::vector<double> cm(static_cast<size_t>(S) * K * k, 0.0), coef(static_cast<size_t>(S) * k, 0.0);
    c->lrc_ritz.assign(static_cast<size_t>(S) * k, 0.0);
    c->lrc_kept.assign(S, 0);
    for (int a = 0; a < S; ++a) {
        const int m = nsteps[a];
        std::vector<double> T(static_cast<size_t>(m) * m, 0.0), ev, Q;
        for (int i = 0; i < m; ++i) {
            T[i * m + i] = alpha[a][i];
            if (i + 1 < m) T[i * m + i + 1] = T[(i + 1) * m + i] = beta[a][i];
        }
        sym_eig(m, T, ev, Q);
        for (int t = 0; t < k && t < m; ++t) {
            const double lam = ev[t];
            c->lrc_ritz[a * k + t] = lam;
            if (!(lam < 1.0) || !(lam > 0.0)) continue;
            coef[a * k + t] = amg ? 1.0 - lam : 1.0 / lam - 1.0;
            c->lrc_kept[a] += 1;
            for (int j = 0; j < m; ++j) cm[(static_cast<size_t>(a) * K + j) * k + t] = Q[j * m + t];
        }
    }
    double* dcm = c->upload(cm.data(), static_cast<int64_t>(cm.size()));
    c->U16 = amg && c->o.precision == MSP_MIXED_BF16;
    c->U32 = mixed(c) && !c->U16;
    if (c->U16) {
        Bf16* U = c->dalloc<Bf16>(n * S * k);
        HIPCHECK(launch_lrc_combine<Bf16>(st, n, S, k, K, C, V, dcm, U));
        c->d_U = U;
    } else if (c->U32) {
        float* U = c->dalloc<float>(n * S * k);
        HIPCHECK(launch_lrc_combine<float>(st, n, S, k, K, C, V, dcm, U));
        c->d_U = U;
    } else {
        double* U = c->dalloc<double>(n * S * k);
        HIPCHECK(launch_lrc_combine<double>(st, n, S, k, K, C, V, dcm, U));
        c->d_U = U;
    }
    c->d_lrc_coef = c->upload(coef.data(), static_cast<int64_t>(coef.size()));
    c->lrc_nb = 512;
    c->d_lrc_part = c->dalloc<double>(static_cast<int64_t>(c->lrc_nb) * S * k * 64);
    c->d_lrc_W = c->dalloc<double>(static_cast<int64_t>(S) * k * 64);
    HIPCHECK(hipStreamSynchronize(st));
    c->dfree(dcm);
    c->dfree(hcoef);
    if (amg) c->dfree(BV);
    c->dfree(V);
}


void build_lrc(msp_ctx* c) {
    const int S = 1 << c->sym.s;
    const int C = next_pow2(S);
    const bool amg = msp::amg(c);
    Work& w = work(c, C);
    w.m = 1;
    hipStream_t st = nullptr;
    double* tmp = w.p;
    auto applyB = [&](const double* x, double* y) {   // y = A_a x per column
        spmm<double>(c, KD_OP, st, C, c->dAinn, x, y, nullptr, 1.0, 0.0, &c->dsig, S, 1);
    };
    auto op = [&](const double* v, const double* bv, double* out) {
        if (amg) {
            precondition_base(c, w, st, bv, out, false);
        } else {
            spmm<double>(c, KD_FSAI, st, C, c->dGfT, v, tmp, nullptr, 1.0, 0.0);
            applyB(tmp, w.z);
            spmm<double>(c, KD_FSAI, st, C, c->dGf, w.z, out, nullptr, 1.0, 0.0);
        }
    };
    lanczos_corrections(c, w, c->sym.n_b, amg, applyB, op);
}

// Corrections of the decoupled Schur blocks for AMGS (eq. (3.11)): LRCFSAI of
// G_S1 toward S_AMG,a = C_1 + Sigma_a - B^T AMG_K B on the interface rows.
void build_schur_lrc(msp_ctx* c) {
    const int S = 1 << c->sym.s;
    const int C = next_pow2(S);
    Work& w = work(c, C);
    w.m = 1;
    hipStream_t st = nullptr;
    const int64_t nG = c->sym.n_b - c->am.nI;
    double* tmp = w.p;
    auto applyB = [&](const double* x, double* y) {   // y = S_AMG,a x per column
        spmm<double>(c, KD_AMGS, st, C, c->dC1, x, y, nullptr, 1.0, 0.0, &c->dsigG, S, 1);
        spmm<double>(c, KD_AMGS, st, C, c->dB, x, w.amgs1, nullptr, 1.0, 0.0);
        vcycle<double>(c, w, st, 0, w.amgs1, w.amgs2);
        spmm<double>(c, KD_AMGS, st, C, c->dBT, w.amgs2, y, y, -1.0, 1.0);
    };
    auto op = [&](const double* v, const double*, double* out) {   // G_S1 S_AMG,a G_S1^T v
        spmm<double>(c, KD_AMGS, st, C, c->dGS1T, v, tmp, nullptr, 1.0, 0.0);
        applyB(tmp, w.z);
        spmm<double>(c, KD_AMGS, st, C, c->dGS1, w.z, out, nullptr, 1.0, 0.0);
    };
    lanczos_corrections(c, w, nG, false, applyB, op);
}

// ====================================================================== numeric re-setup on the device

static RfPat upload_pat(msp_ctx* c, const Csr& M) {
    if (M.nnz() >= (int64_t(1) << 31)) throw Error(MSP_ERR_UNSUPPORTED, "matrix too large for 32-bit indices");
    RfPat P;
    P.nr = M.nr;
    P.nnz = M.nnz();
    std::vector<int32_t> rp(M.nr + 1);
    for (int64_t i = 0; i <= M.nr; ++i) rp[i] = static_cast<int32_t>(M.rp[i]);
    P.rp = c->upload(rp.data(), M.nr + 1);
    P.ci = c->upload(M.ci.data(), P.nnz);
    return P;
}

static RfPat dev_pat(const DevCsr& D) {
    RfPat P;
    P.rp = D.rp;
    P.ci = D.ci;
    P.nr = D.nr;
    P.nnz = D.nnz;
    return P;
}

// FSAI workspace offsets of G's rows: k^2 + k doubles per row
static int64_t* fsai_offsets(msp_ctx* c, const Csr& G, int64_t* total) {
    std::vector<int64_t> off(G.nr + 1, 0);
    for (int64_t i = 0; i < G.nr; ++i) {
        const int64_t k = G.rp[i + 1] - G.rp[i];
        off[i + 1] = off[i] + k * k + k;
    }
    *total = off[G.nr];
    return c->upload(off.data(), G.nr + 1);
}

// Compact outer-diagonal values (upload_outer's layout) <- sigma entries
static std::vector<int64_t> outer_sources(const std::vector<double>& dense, int64_t rows, int S,
                                          const std::vector<int64_t>& base_of_row) {
    std::vector<int64_t> src;
    for (int64_t i = 0; i < rows; ++i) {
        bool any = false;
        for (int a = 0; a < S; ++a) any |= dense[i * S + a] != 0.0;
        if (!any) continue;
        for (int a = 0; a < S; ++a) src.push_back(base_of_row[i] * S + a);
    }
    return src;
}

static void refresh_build(msp_ctx* c) {
    // MSP_SETUP_LOG set (non-empty, not "0"): seconds per phase to stderr
    const char* logv = std::getenv("MSP_SETUP_LOG");
    const bool tlog = logv && *logv && std::strcmp(logv, "0") != 0;
    auto clk = std::chrono::steady_clock::now();
    auto lap = [&](const char* what, long l) {
        if (!tlog) return;
        const auto t = std::chrono::steady_clock::now();
        std::fprintf(stderr, "msp re-setup structure: %s %ld %.3f s\n", what, l,
                     std::chrono::duration<double>(t - clk).count());
        clk = t;
    };
    std::unique_ptr<RefreshState> R(new RefreshState());
    const int S = 1 << c->sym.s;
    const int64_t nb = c->sym.n_b;
    if (static_cast<int64_t>(c->sym.inn_src.size()) != c->sym.Ainn.nnz())
        throw Error(MSP_ERR_UNSUPPORTED, "no source map of the setup matrix");
    R->inn_src = c->upload(c->sym.inn_src.data(), static_cast<int64_t>(c->sym.inn_src.size()));
    if (S > 1) R->out_src = c->upload(c->sym.out_src.data(), static_cast<int64_t>(c->sym.out_src.size()));
    R->sigma = c->dalloc<double>(nb * S);
    {
        std::vector<int64_t> ident(nb);
        std::iota(ident.begin(), ident.end(), int64_t(0));
        const std::vector<int64_t> ds = outer_sources(c->sym.sigma, nb, S, ident);
        if (static_cast<int64_t>(ds.size()) != c->dsig.carried * S) throw Error(MSP_ERR_ARG, "outer diagonal layout");
        R->ndsig = static_cast<int64_t>(ds.size());
        if (R->ndsig) R->dsig_src = c->upload(ds.data(), R->ndsig);
    }
    R->err = c->dalloc<int>(1);
    // Alg. 2 redone for the new values (not for a domain of copies, whose split is replicated);
    // level 1's standard split (priorities: strong dependants, then hash) as well
    auto make_check = [&](SplitCheck& K, const Csr& A, const RfPat& pat, int d, uint64_t lev_bits,
                          const std::vector<int8_t>& cand, const std::vector<int8_t>& cf, bool pmis) {
        const int64_t n = A.nr;
        const std::vector<int64_t> tm = transpose_map(A);   // operator patterns here are symmetric
        std::vector<uint64_t> pri(n);
        std::vector<int8_t> st0(n);
        for (int64_t i = 0; i < n; ++i) {
            pri[i] = splitmix64(c->o.seed ^ lev_bits ^ static_cast<uint64_t>(i));
            st0[i] = cand[i] ? 0 : 3;
        }
        K.A = pat;
        K.d = d;
        K.tmap = c->upload(tm.data(), static_cast<int64_t>(tm.size()));
        K.pri = c->upload(pri.data(), n);
        K.state_init = c->upload(st0.data(), n);
        K.cf = c->upload(cf.data(), n);
        K.smask = c->dalloc<int8_t>(A.nnz());
        K.tmask = c->dalloc<int8_t>(A.nnz());
        K.state = c->dalloc<int8_t>(n);
        if (pmis) K.lam = c->dalloc<int32_t>(n);
        K.on = true;
    };
    if (cycle(c) && c->o.pc != MSP_PC_AMGS) {
        R->left = c->dalloc<int>(1);
        R->diff = c->dalloc<unsigned long long>(1);
        if (!c->copies && c->o.dist <= 3) {
            std::vector<int8_t> cand(nb);
            for (int64_t i = 0; i < nb; ++i) cand[i] = c->sym.iface[i] ? 0 : 1;
            make_check(R->sc0, c->sym.Ainn, dev_pat(c->dAinn), c->o.dist, 0, cand, c->hier.lev[0].cf, false);
        }
        if (c->hier.lev.size() > 2) {
            const HostLevel& H1 = c->hier.lev[1];
            make_check(R->sc1, H1.A, dev_pat(c->dl[1].A), 1, uint64_t(1) << 40, std::vector<int8_t>(H1.A.nr, 1),
                       H1.cf, true);
        }
    }
    lap("sources and split checks", -1);
    R->part = c->dalloc<double>(2 * R->nbp);
    R->dots = c->dalloc<double>(2);
    if (cycle(c)) {
        const size_t L = c->hier.lev.size();
        R->lev.resize(L);
        int64_t work = 0, maxn = 0;
        for (size_t l = 0; l < L; ++l) {
            const HostLevel& H = c->hier.lev[l];
            RfLevel& F = R->lev[l];
            F.n = H.A.nr;
            maxn = std::max(maxn, F.n);
            F.A = l + 1 < L ? dev_pat(c->dl[l].A) : upload_pat(c, H.A);
            F.a = c->dalloc<double>(H.A.nnz());
            if (l + 1 == L) break;
            const DevLevel& D = c->dl[l];
            if (!D.M.rp) throw Error(MSP_ERR_UNSUPPORTED, "the re-setup needs the explicit smoother");
            F.G = upload_pat(c, H.G);
            F.GT = upload_pat(c, H.GT);
            const std::vector<int64_t> gts = transpose_map(H.G);
            F.gt_src = c->upload(gts.data(), static_cast<int64_t>(gts.size()));
            F.M = dev_pat(D.M);
            F.P = dev_pat(D.P);
            F.R = dev_pat(D.R);
            const std::vector<int64_t> rs = transpose_map(H.P);
            F.r_src = c->upload(rs.data(), static_cast<int64_t>(rs.size()));
            lap("patterns and transposes, level", static_cast<long>(l));
            const int steps = l == 0 ? c->o.jacobi0 : c->o.jacobi;
            const std::vector<Csr> Ws = interpolation_patterns(H.A, H.cf, steps);
            lap("interpolation patterns, level", static_cast<long>(l));
            for (const Csr& W : Ws) {
                F.W.push_back(upload_pat(c, W));
                F.w.push_back(c->dalloc<double>(W.nnz()));
            }
            const Csr& WL = Ws.back();
            F.nf = WL.nr;
            F.afc = c->dalloc<double>(std::max<int64_t>(1, [&] {
                int64_t mx = 0;
                for (const Csr& W : Ws) mx = std::max(mx, W.nnz());
                return mx;
            }()));
            F.hasf = c->dalloc<int8_t>(std::max<int64_t>(1, [&] {
                int64_t mx = 0;
                for (const Csr& W : Ws) mx = std::max(mx, W.nnz());
                return mx;
            }()));
            std::vector<int32_t> fidx, cnum(F.n, -1), fnum(F.n, -1);
            int32_t nc = 0, nf = 0;
            for (int64_t i = 0; i < F.n; ++i) {
                if (H.cf[i]) cnum[i] = nc++;
                else {
                    fnum[i] = nf++;
                    fidx.push_back(static_cast<int32_t>(i));
                }
            }
            std::vector<int32_t> pmap(H.P.nnz(), 0);
            for (int64_t i = 0; i < F.n; ++i) {
                if (H.cf[i]) continue;
                const int32_t r = fnum[i];
                for (int64_t e = H.P.rp[i]; e < H.P.rp[i + 1]; ++e) {
                    const int32_t* b = WL.ci.data() + WL.rp[r];
                    const int32_t* en = WL.ci.data() + WL.rp[r + 1];
                    const int32_t* f = std::lower_bound(b, en, H.P.ci[e]);
                    if (f == en || *f != H.P.ci[e]) throw Error(MSP_ERR_ARG, "interpolation pattern outside its steps");
                    pmap[e] = static_cast<int32_t>(f - WL.ci.data());
                }
            }
            F.pmap = c->upload(pmap.data(), static_cast<int64_t>(pmap.size()));
            F.fidx = c->upload(fidx.data(), std::max<int64_t>(1, nf));
            F.cnum = c->upload(cnum.data(), F.n);
            F.fnum = c->upload(fnum.data(), F.n);
            F.cf = c->upload(H.cf.data(), F.n);
            lap("interpolation maps, level", static_cast<long>(l));
            F.AP = upload_pat(c, spgemm(H.A, H.P));
            lap("AP pattern, level", static_cast<long>(l));
            int64_t wk = 0;
            F.woff = fsai_offsets(c, H.G, &wk);
            lap("FSAI offsets, level", static_cast<long>(l));
            work = std::max(work, wk);
            std::vector<double> v0(F.n);
            double nrm = 0.0;
            for (int64_t i = 0; i < F.n; ++i) {
                v0[i] = unit_centered(c->o.seed ^ static_cast<uint64_t>(i));
                nrm += v0[i] * v0[i];
            }
            nrm = std::sqrt(nrm);
            for (auto& x : v0) x /= nrm;
            F.v0 = c->upload(v0.data(), F.n);
            F.g = c->dalloc<double>(H.G.nnz());
            F.gt = c->dalloc<double>(H.G.nnz());
            F.m = c->dalloc<double>(H.M.nnz());
            F.p = c->dalloc<double>(H.P.nnz());
            F.r = c->dalloc<double>(H.P.nnz());
            F.ap = c->dalloc<double>(F.AP.nnz);
        }
        R->work = c->dalloc<double>(std::max<int64_t>(1, work));
        R->emin_steps = c->o.emin_steps;
        if (R->emin_steps > 0) {
            int64_t mp = 1;
            for (size_t l = 0; l + 1 < L; ++l) mp = std::max(mp, c->hier.lev[l].P.nnz());
            for (double*& e : R->em) e = c->dalloc<double>(mp);
        }
        R->t1 = c->dalloc<double>(maxn);
        R->t2 = c->dalloc<double>(maxn);
        R->t3 = c->dalloc<double>(maxn);
        const int64_t nL = c->hier.lev.back().A.nr;
        const int Sd = c->sub ? S : 1;
        R->dense = c->dalloc<double>(static_cast<int64_t>(Sd) * nL * nL);
        R->rowk = c->dalloc<double>(static_cast<int64_t>(Sd) * nL);
        R->colk = c->dalloc<double>(static_cast<int64_t>(Sd) * nL);
        if (c->sub) {
            R->shared1 = c->dalloc<double>(c->hier.lev[1].A.nnz());
            R->sub_g.assign(L, nullptr);
            for (size_t l = 1; l + 1 < L; ++l) R->sub_g[l] = c->dalloc<double>(c->hier.lev[l].G.nnz() * S);
            if (L > 2) R->sub_a1 = c->dalloc<double>(c->hier.lev[1].A.nnz() * S);
        }
        if (c->sub && L > 2) {
            R->sets = c->dalloc<double>(c->hier.lev.back().A.nnz() * S);
            // interface coarse points: their A_1 diagonal entries and base cells
            const HostLevel& L0 = c->hier.lev[0];
            const Csr& A1 = c->hier.lev[1].A;
            std::vector<int64_t> diag, base, rowbase(A1.nr, -1);
            int64_t j = 0;
            for (int64_t i = 0; i < L0.A.nr; ++i) {
                if (!L0.cf[i]) continue;
                rowbase[j] = i;
                if (c->sym.iface[i]) {
                    const int32_t* b = A1.ci.data() + A1.rp[j];
                    const int32_t* e = A1.ci.data() + A1.rp[j + 1];
                    const int32_t* f = std::lower_bound(b, e, static_cast<int32_t>(j));
                    if (f == e || *f != j) throw Error(MSP_ERR_ARG, "missing diagonal in the reduced operator");
                    diag.push_back(f - A1.ci.data());
                    base.push_back(i);
                }
                ++j;
            }
            R->ns1 = static_cast<int64_t>(diag.size());
            if (R->ns1) {
                R->s1_diag = c->upload(diag.data(), R->ns1);
                R->s1_base = c->upload(base.data(), R->ns1);
            }
            // level-1 compact outer diagonal (upload_all's s1 layout)
            std::vector<double> s1(static_cast<size_t>(A1.nr) * S, 0.0);
            for (int64_t q = 0; q < A1.nr; ++q)
                if (rowbase[q] >= 0 && c->sym.iface[rowbase[q]])
                    for (int a = 0; a < S; ++a) s1[q * S + a] = c->sym.sigma[rowbase[q] * S + a];
            const std::vector<int64_t> d1 = outer_sources(s1, A1.nr, S, rowbase);
            if (static_cast<int64_t>(d1.size()) != c->dsig1.carried * S) throw Error(MSP_ERR_ARG, "level-1 outer layout");
            R->ndsig1 = static_cast<int64_t>(d1.size());
            if (R->ndsig1) R->dsig1_src = c->upload(d1.data(), R->ndsig1);
        } else if (c->sub) {   // two levels: the coarsest operators are A_1,a themselves
            R->sets = c->dalloc<double>(c->hier.lev.back().A.nnz() * S);
            const HostLevel& L0 = c->hier.lev[0];
            const Csr& A1 = c->hier.lev[1].A;
            std::vector<int64_t> diag, base;
            int64_t j = 0;
            for (int64_t i = 0; i < L0.A.nr; ++i) {
                if (!L0.cf[i]) continue;
                if (c->sym.iface[i]) {
                    const int32_t* b = A1.ci.data() + A1.rp[j];
                    const int32_t* e = A1.ci.data() + A1.rp[j + 1];
                    const int32_t* f = std::lower_bound(b, e, static_cast<int32_t>(j));
                    if (f == e || *f != j) throw Error(MSP_ERR_ARG, "missing diagonal in the reduced operator");
                    diag.push_back(f - A1.ci.data());
                    base.push_back(i);
                }
                ++j;
            }
            R->ns1 = static_cast<int64_t>(diag.size());
            if (R->ns1) {
                R->s1_diag = c->upload(diag.data(), R->ns1);
                R->s1_base = c->upload(base.data(), R->ns1);
            }
        }
    } else if (c->o.pc == MSP_PC_FSAI) {
        R->gfp = dev_pat(c->dGf);
        R->gftp = dev_pat(c->dGfT);
        const std::vector<int64_t> m = transpose_map(c->Gf);
        R->gft_src = c->upload(m.data(), static_cast<int64_t>(m.size()));
        int64_t wk = 0;
        R->gf_woff = fsai_offsets(c, c->Gf, &wk);
        R->work = c->dalloc<double>(std::max<int64_t>(1, wk));
    }
    lap("rest", -1);
    c->rf = std::move(R);
}

// One level's FSAI, damping and explicit smoother from the values in F.a.
static void refresh_smoother(RefreshState& R, RfLevel& F, hipStream_t st) {
    HIPCHECK(launch_fsai(st, F.n, F.A.rp, F.A.ci, F.a, F.G.rp, F.G.ci, F.g, F.woff, R.work, R.err));
    HIPCHECK(launch_gather(st, F.G.nnz, F.gt_src, F.g, F.gt));
    // omega = 4 / (3 lambda), lambda from 20 power iterations on G A G^T
    HIPCHECK(hipMemcpyAsync(R.t3, F.v0, sizeof(double) * F.n, hipMemcpyDeviceToDevice, st));
    for (int it = 0; it < 20; ++it) {
        HIPCHECK(launch_spmv(st, F.n, F.GT.rp, F.GT.ci, F.gt, R.t3, R.t1, F.GT.nnz));
        HIPCHECK(launch_spmv(st, F.n, F.A.rp, F.A.ci, F.a, R.t1, R.t2, F.A.nnz));
        HIPCHECK(launch_spmv(st, F.n, F.G.rp, F.G.ci, F.g, R.t2, R.t1, F.G.nnz));
        HIPCHECK(launch_power_dots(st, F.n, R.t3, R.t1, R.part, R.nbp, R.dots));
        HIPCHECK(launch_normalise(st, F.n, R.t1, R.dots, R.t3));
    }
    double dots[2];
    HIPCHECK(hipMemcpyAsync(dots, R.dots, sizeof(dots), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    F.omega = 4.0 / (3.0 * dots[0]);
    HIPCHECK(launch_spgemm_masked(st, F.n, F.M.nnz, F.GT.rp, F.GT.ci, F.gt, F.G.rp, F.G.ci, F.g, F.M.rp, F.M.ci, F.m));
    HIPCHECK(launch_scale(st, F.M.nnz, F.m, F.omega));
}

// Interpolation (the Jacobi steps, the kept pattern, the row rescaling), R, and next = R (A P).
// Energy minimisation of a level's interpolation, as the setup does it:
// projected, Jacobi-preconditioned CG on tr(P^T A P) with P's pattern and row
// sums fixed.  P's C rows are unit rows, so on the F rows the masked product
// A P on P's pattern is A_FF W + A_FC (the half gradient), and with the C rows
// zero (the search directions) it is A_FF D.
static void refresh_emin(RefreshState& R, RfLevel& F, hipStream_t st) {
    const int64_t m = F.P.nnz, n = F.n;
    double *g = R.em[0], *r = R.em[1], *z = R.em[2], *p = R.em[3], *q = R.em[4], *dinv = R.em[5];
    auto dot = [&](const double* a, const double* b) {
        HIPCHECK(launch_power_dots(st, m, a, b, R.part, R.nbp, R.dots));
        double h[2];
        HIPCHECK(hipMemcpyAsync(h, R.dots, sizeof(h), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        return h[0];
    };
    HIPCHECK(launch_emin_dinv(st, n, F.A.rp, F.A.ci, F.a, F.P.rp, dinv));
    HIPCHECK(launch_spgemm_masked(st, n, m, F.A.rp, F.A.ci, F.a, F.P.rp, F.P.ci, F.p, F.P.rp, F.P.ci, g));
    HIPCHECK(launch_emin_project(st, n, F.P.rp, F.cf, g, -1.0, r));
    HIPCHECK(launch_mul(st, m, dinv, r, z));
    HIPCHECK(hipMemcpyAsync(p, z, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    double rz = dot(r, z);
    for (int it = 0; it < R.emin_steps; ++it) {
        if (!(rz > 0.0)) break;
        HIPCHECK(launch_spgemm_masked(st, n, m, F.A.rp, F.A.ci, F.a, F.P.rp, F.P.ci, p, F.P.rp, F.P.ci, g));
        HIPCHECK(launch_emin_project(st, n, F.P.rp, F.cf, g, 1.0, q));
        const double pq = dot(p, q);
        if (!(pq > 0.0)) break;
        HIPCHECK(launch_emin_step(st, m, rz / pq, p, q, dinv, F.p, r, z));
        const double rz_new = dot(r, z);
        HIPCHECK(launch_emin_dir(st, m, rz_new / rz, z, p));
        rz = rz_new;
    }
}

static void refresh_transfer(RefreshState& R, RfLevel& F, double* next, const RfPat& nextpat,
                             hipStream_t st) {
    for (size_t t = 0; t < F.W.size(); ++t) {
        const bool first = t == 0;
        HIPCHECK(launch_interp_step(st, F.nf, F.fidx, F.A.rp, F.A.ci, F.a, F.cf, F.cnum, F.fnum,
                                    first ? nullptr : F.W[t - 1].rp, first ? nullptr : F.W[t - 1].ci,
                                    first ? nullptr : F.w[t - 1], F.W[t].rp, F.W[t].ci, F.w[t], F.afc, F.hasf, R.err));
    }
    HIPCHECK(launch_interp_finish(st, F.n, F.cf, F.A.rp, F.A.ci, F.a, F.w.back(), F.P.rp, F.pmap, F.p));
    if (R.emin_steps > 0) refresh_emin(R, F, st);
    HIPCHECK(launch_gather(st, F.R.nnz, F.r_src, F.p, F.r));
    HIPCHECK(launch_spgemm_masked(st, F.n, F.AP.nnz, F.A.rp, F.A.ci, F.a, F.P.rp, F.P.ci, F.p, F.AP.rp, F.AP.ci, F.ap));
    HIPCHECK(launch_spgemm_masked(st, nextpat.nr, nextpat.nnz, F.R.rp, F.R.ci, F.r, F.AP.rp, F.AP.ci, F.ap,
                                  nextpat.rp, nextpat.ci, next));
}

// FP32 copy of a device matrix's values (mixed modes)
static void refresh_f32(hipStream_t st, DevCsr& D) {
    if (D.v32) HIPCHECK((launch_cast<float, double>(st, D.nnz * D.vs, D.v64, D.v32)));
}

// Points of a level whose C/F decision a fresh setup of these values would
// take differently (the strength of connection, then the distance-d
// independent set in rounds); -1 when the check is off or did not finish.
static int64_t split_drift(RefreshState& R, SplitCheck& K, const double* v, double theta, hipStream_t st) {
    if (!K.on) return -1;
    const int64_t n = K.A.nr;
    HIPCHECK(launch_split_strength(st, n, K.A.nnz, K.A.rp, K.A.ci, v, theta, K.tmap, K.smask, K.tmask));
    if (K.lam) {
        HIPCHECK(hipMemsetAsync(K.lam, 0, sizeof(int32_t) * n, st));
        HIPCHECK(launch_strong_dependants(st, n, K.A.rp, K.A.ci, K.smask, K.lam));
    }
    HIPCHECK(hipMemcpyAsync(K.state, K.state_init, n, hipMemcpyDeviceToDevice, st));
    for (int round = 0; round < 4096; ++round) {
        HIPCHECK(hipMemsetAsync(R.left, 0, sizeof(int), st));
        HIPCHECK(launch_mis_round(st, n, K.d, K.A.rp, K.A.ci, K.tmask, K.lam, K.pri, K.state, R.left));
        int left = 0;
        HIPCHECK(hipMemcpyAsync(&left, R.left, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        if (left == 0) {
            unsigned long long diff = 0;
            HIPCHECK(hipMemsetAsync(R.diff, 0, sizeof(diff), st));
            HIPCHECK(launch_split_diff(st, n, K.state, K.cf, R.diff));
            HIPCHECK(hipMemcpyAsync(&diff, R.diff, sizeof(diff), hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
            return static_cast<int64_t>(diff);
        }
    }
    return -1;
}

// One shared level's values (smoother, transfers, the next level's operator).
static void refresh_shared_level(RefreshState& R, size_t l, hipStream_t st) {
    RfLevel& F = R.lev[l];
    refresh_smoother(R, F, st);
    refresh_transfer(R, F, R.lev[l + 1].a, R.lev[l + 1].A, st);
}

void refresh_device(msp_ctx* c, const double* d_val, hipStream_t st) {
    if (!d_val) throw Error(MSP_ERR_ARG, "null values");
    if (!c->on_device) throw Error(MSP_ERR_ARG, "the context has no device setup");
    if (c->o.pc == MSP_PC_AMGS) throw Error(MSP_ERR_UNSUPPORTED, "the re-setup of AMGS");
    if (c->o.precision == MSP_MIXED_FP32_BF16G) throw Error(MSP_ERR_UNSUPPORTED, "the re-setup of the BF16-G variant");
    HIPCHECK(hipSetDevice(c->device));
    const char* logv = std::getenv("MSP_SETUP_LOG");
    const bool tlog = logv && *logv && std::strcmp(logv, "0") != 0;
    auto clk = std::chrono::steady_clock::now();
    auto lap = [&](const char* what) {
        if (!tlog) return;
        HIPCHECK(hipStreamSynchronize(st));
        const auto t = std::chrono::steady_clock::now();
        std::fprintf(stderr, "msp re-setup: %s %.3f s\n", what, std::chrono::duration<double>(t - clk).count());
        clk = t;
    };
    if (!c->rf) refresh_build(c);
    lap("structure");
    RefreshState& R = *c->rf;
    c->values_invalid = true;   // until this re-setup completes
    const int S = 1 << c->sym.s;
    const int64_t nb = c->sym.n_b;
    HIPCHECK(hipMemsetAsync(R.err, 0, sizeof(int), st));
    // A_inn (operator and level 0) and the outer diagonal from the caller's values
    HIPCHECK(launch_gather(st, c->dAinn.nnz, R.inn_src, d_val, c->dAinn.v64));
    HIPCHECK(launch_outer_sigma(st, nb, S, R.out_src, d_val, R.sigma));
    if (R.ndsig) HIPCHECK(launch_gather(st, R.ndsig, R.dsig_src, R.sigma, const_cast<double*>(c->dsig.d.val)));
    c->stats.split_drift = split_drift(R, R.sc0, c->dAinn.v64, c->o.theta, st);
    c->stats.split_drift1 = -1;
    if (cycle(c)) {
        const size_t L = R.lev.size();
        HIPCHECK(hipMemcpyAsync(R.lev[0].a, c->dAinn.v64, sizeof(double) * c->dAinn.nnz, hipMemcpyDeviceToDevice,
                                st));
        // shared levels: all of them for the shared cycle, the reduction level for
        // the per-subsystem one (its shared levels below are recomputed only when
        // the host copy is asked for)
        const size_t shared_to = c->sub ? 1 : L - 1;
        for (size_t l = 0; l < shared_to; ++l) {
            RfLevel& F = R.lev[l];
            refresh_shared_level(R, l, st);
            DevLevel& D = c->dl[l];
            D.omega = F.omega;
            auto put = [&](DevCsr& M, const double* v) {
                HIPCHECK(hipMemcpyAsync(M.v64, v, sizeof(double) * M.nnz, hipMemcpyDeviceToDevice, st));
            };
            put(D.A, F.a);
            put(D.M, F.m);
            put(D.P, F.p);
            put(D.R, F.r);
        }
        // level 1's split for the shared A_1 of these values (per-subsystem mode: before the
        // subsystems overwrite that buffer)
        c->stats.split_drift1 = split_drift(R, R.sc1, R.lev[1].a, c->o.theta, st);
        const int64_t nL = c->hier.lev.back().A.nr;
        if (!c->sub) {
            RfLevel& FL = R.lev[L - 1];
            HIPCHECK(launch_dense_inverse(st, nL, 1, FL.A.rp, FL.A.ci, FL.a, R.dense, R.rowk, R.colk));
            HIPCHECK(hipMemcpyAsync(c->d_cinv, R.dense, sizeof(double) * nL * nL, hipMemcpyDeviceToDevice, st));
        } else {
            // A_1 shared values and the level-1 outer diagonal (three or more levels)
            if (L > 2)
                HIPCHECK(hipMemcpyAsync(c->dl[1].A.v64, R.lev[1].a, sizeof(double) * c->dl[1].A.nnz,
                                        hipMemcpyDeviceToDevice, st));
            if (R.ndsig1)
                HIPCHECK(launch_gather(st, R.ndsig1, R.dsig1_src, R.sigma, const_cast<double*>(c->dsig1.d.val)));
            const int64_t n1 = R.lev[1].A.nnz;
            HIPCHECK(hipMemcpyAsync(R.shared1, R.lev[1].a, sizeof(double) * n1, hipMemcpyDeviceToDevice, st));
            for (int a = 0; a < S; ++a) {
                HIPCHECK(hipMemcpyAsync(R.lev[1].a, R.shared1, sizeof(double) * n1, hipMemcpyDeviceToDevice, st));
                if (R.ns1) HIPCHECK(launch_add_sigma(st, R.ns1, R.s1_diag, R.s1_base, R.sigma, S, a, R.lev[1].a));
                if (L > 2) HIPCHECK(launch_strided_copy(st, n1, R.lev[1].a, 1, 0, R.sub_a1, S, a));
                for (size_t l = 1; l + 1 < L; ++l) {
                    RfLevel& F = R.lev[l];
                    refresh_smoother(R, F, st);
                    HIPCHECK(launch_strided_copy(st, F.G.nnz, F.g, 1, 0, R.sub_g[l], S, a));
                    refresh_transfer(R, F, R.lev[l + 1].a, R.lev[l + 1].A, st);
                    DevLevel& D = c->dl[l];
                    c->subv.omega[l][a] = F.omega;
                    HIPCHECK(launch_strided_copy(st, F.P.nnz, F.p, 1, 0, D.P.v64, S, a));
                    HIPCHECK(launch_strided_copy(st, F.R.nnz, F.r, 1, 0, D.R.v64, S, a));
                    HIPCHECK(launch_strided_copy(st, F.M.nnz, F.m, 1, 0, D.M.v64, S, a));
                    if (l + 1 < L - 1)
                        HIPCHECK(launch_strided_copy(st, R.lev[l + 1].A.nnz, R.lev[l + 1].a, 1, 0, c->dl[l + 1].A.v64, S,
                                                     a));
                }
                HIPCHECK(launch_strided_copy(st, R.lev[L - 1].A.nnz, R.lev[L - 1].a, 1, 0, R.sets, S, a));
            }
            const RfLevel& FL = R.lev[L - 1];
            HIPCHECK(launch_dense_inverse(st, nL, S, FL.A.rp, FL.A.ci, R.sets, R.dense, R.rowk, R.colk));
            if (c->d_cinv32) {
                const int64_t ld = dense_sets_ld(nL, 4);
                HIPCHECK(launch_dense_to_f32(st, S, nL, ld, R.dense, c->d_cinv32));
            } else {
                HIPCHECK(hipMemcpyAsync(c->d_cinv, R.dense, sizeof(double) * S * nL * nL, hipMemcpyDeviceToDevice, st));
            }
        }
        lap("levels");
        // FP32 copies of the level matrices (mixed modes) and the sliced forms in use
        for (DevLevel& D : c->dl)
            for (DevCsr* M : {&D.A, &D.P, &D.R, &D.M}) {
                refresh_f32(st, *M);
                refresh_sells(c, *M, st);
            }
    } else if (c->o.pc == MSP_PC_FSAI) {
        HIPCHECK(launch_fsai(st, nb, c->dAinn.rp, c->dAinn.ci, c->dAinn.v64, R.gfp.rp, R.gfp.ci, c->dGf.v64, R.gf_woff,
                             R.work, R.err));
        HIPCHECK(launch_gather(st, R.gftp.nnz, R.gft_src, c->dGf.v64, c->dGfT.v64));
    }
    refresh_sells(c, c->dAinn, st);
    lap("copies and sliced forms");
    int err = 0;
    HIPCHECK(hipMemcpyAsync(&err, R.err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    c->host_stale = true;   // the host copy is fetched when something reads it (sync_host)
    R.shared_stale = c->sub;
    if (err & 2) throw Error(MSP_ERR_NOT_SPD, "re-setup: an FSAI block of the new matrix is not positive definite");
    if (err) throw Error(MSP_ERR_ARG, "re-setup: an interpolation weight left its kept pattern");
    // low-rank corrections of the new operators
    if (c->lrc_k > 0) {
        for (void* q : {c->d_U, static_cast<void*>(c->d_lrc_coef), static_cast<void*>(c->d_lrc_part),
                        static_cast<void*>(c->d_lrc_W)})
            if (q) c->dfree(q);
        c->d_U = nullptr;
        c->d_lrc_coef = c->d_lrc_part = c->d_lrc_W = nullptr;
        build_lrc(c);
        lap("corrections");
    }
    HIPCHECK(hipDeviceSynchronize());
    c->values_invalid = false;
}

// Host copy of every value after a device re-setup (exports, and sliced forms
// the autotuner builds later, read it).  With per-subsystem values the shared
// levels below the reduction level are recomputed here first: the solve does
// not use them.
void sync_host(msp_ctx* c) {
    if (!c->host_stale || !c->rf) return;
    RefreshState& R = *c->rf;
    HIPCHECK(hipSetDevice(c->device));
    hipStream_t st = nullptr;
    const int S = 1 << c->sym.s;
    const int64_t nb = c->sym.n_b;
    auto down = [&](std::vector<double>& h, const double* d, int64_t count) {
        h.resize(count);
        HIPCHECK(hipMemcpy(h.data(), d, sizeof(double) * count, hipMemcpyDeviceToHost));
    };
    down(c->sym.Ainn.v, c->dAinn.v64, c->dAinn.nnz);
    down(c->sym.sigma, R.sigma, nb * S);
    if (cycle(c)) {
        const size_t L = R.lev.size();
        if (c->sub) {
            // per-subsystem values first: the shared recomputation below reuses the level buffers
            for (size_t l = 1; l + 1 < L; ++l) {
                const DevLevel& D = c->dl[l];
                down(c->subv.P[l], D.P.v64, D.P.nnz * S);
                down(c->subv.R[l], D.R.v64, D.R.nnz * S);
                down(c->subv.M[l], D.M.v64, D.M.nnz * S);
                down(c->subv.G[l], R.sub_g[l], R.lev[l].G.nnz * S);
                if (l >= 2) down(c->subv.A[l], D.A.v64, D.A.nnz * S);
            }
            if (L > 2) down(c->subv.A[1], R.sub_a1, R.lev[1].A.nnz * S);
            down(c->subv.A[L - 1], R.sets, c->hier.lev.back().A.nnz() * S);
            down(c->subv.coarse_inv, R.dense, static_cast<int64_t>(S) * c->nL * c->nL);
            if (R.shared_stale) {
                HIPCHECK(hipMemcpy(R.lev[1].a, R.shared1, sizeof(double) * R.lev[1].A.nnz, hipMemcpyDeviceToDevice));
                for (size_t l = 1; l + 1 < L; ++l) {
                    refresh_shared_level(R, l, st);
                    c->hier.lev[l].omega = R.lev[l].omega;
                }
                HIPCHECK(hipStreamSynchronize(st));
                R.shared_stale = false;
            }
        } else {
            down(c->hier.coarse_inv, R.dense, c->nL * c->nL);
        }
        for (size_t l = 0; l < L; ++l) {
            HostLevel& H = c->hier.lev[l];
            const RfLevel& F = R.lev[l];
            down(H.A.v, F.a, H.A.nnz());
            if (l + 1 == L) break;
            down(H.G.v, F.g, H.G.nnz());
            down(H.GT.v, F.gt, H.GT.nnz());
            down(H.M.v, F.m, H.M.nnz());
            down(H.P.v, F.p, H.P.nnz());
            down(H.R.v, F.r, H.R.nnz());
            H.omega = F.omega;
        }
    } else if (c->o.pc == MSP_PC_FSAI) {
        down(c->Gf.v, c->dGf.v64, c->dGf.nnz);
    }
    c->host_stale = false;
}

}  // namespace msp
