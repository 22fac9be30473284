// Host-callable launchers of the HIP kernels (kernels.hip).  C is the padded
// column count of the multivectors (a power of two, 1..64).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

namespace msp {

// bfloat16 storage (upper 16 bits of an IEEE binary32), used for matrix values
// and, in the MSP_MIXED_BF16 mode, for the V-cycle multivectors
struct Bf16 {
    uint16_t bits;
};

// Arithmetic type of a storage type: multivectors stored in bfloat16 are
// loaded into FP32 registers and accumulated in FP32.
template <typename T>
struct Acc {
    using type = T;
};
template <>
struct Acc<Bf16> {
    using type = float;
};
template <typename T>
using acc_t = typename Acc<T>::type;

// Per-subsystem outer diagonal of the decoupled operators (eq. (2.14)), kept
// only for the rows that carry one (the interface): idx[row] = -1 for a row
// without it, else its row q in val, val[q * S + a] = sigma_a.  idx == nullptr:
// no outer term.
struct OuterDiag {
    const int32_t* idx;
    const double* val;
};

// Sliced-ELL form of an FP64 matrix with one group per row (the operator):
// ci == nullptr means the CSR form is used.
struct SellRef {
    const int64_t* off;
    const int32_t* wid;
    const int32_t* ci;
    const double* va;
};

// Columns per lane of an n x C multivector of elem_bytes elements: 16-byte
// vectors for FP32/FP64; 8-byte vectors (4 columns) for bfloat16, so that a
// lane's columns stay within one subsystem for m = 4 as they do in FP32.
constexpr int lane_width(int elem_bytes) { return (elem_bytes == 2 ? 8 : 16) / elem_bytes; }

// Every launcher of the solve's kernels takes an optional gate (device.hpp,
// gate_closed): the batched solve passes its system's active flags, so the
// kernels of a converged system return at once.
//
// Y = alpha (A X [+ outer diagonal]) + beta Z with matrix values of type TV
// (TV = T, or Bf16 with T = float) and multivectors of type T.  vs > 1: the
// matrix holds vs interleaved value sets (entry k of set a at va[k*vs + a],
// FP64/FP32 values only) and column c uses set min(c / m, vs - 1).
// wide (one value set only): 16-byte lanes where they differ from the default
// (bfloat16: 8 columns per lane), see spmm_has_wide.
template <typename T, typename TV>
hipError_t launch_spmm(hipStream_t st, int C, int64_t n, const int32_t* rp, const int32_t* ci, const TV* va,
                       const T* X, T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta, OuterDiag sigma, int S, int m,
                       int vs, bool wide = false, const int* gate = nullptr);
bool spmm_has_wide(int C, int elem_bytes);
// Same product for long rows: G lane groups share each row (G a power of two).
template <typename T, typename TV>
hipError_t launch_spmm_split(hipStream_t st, int C, int G, int64_t n, const int32_t* rp, const int32_t* ci,
                             const TV* va, const T* X, T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta, int vs, int m,
                             OuterDiag sigma, int S, const int* gate = nullptr);
// The same product on the sliced-ELL form (sell.hip): rows split into G
// virtual rows (G = 1, 2, 4, 8, 16), slices of 64 virtual rows with width
// wid[s] stored column-major from slot off[s] (column -1 = padding), values
// with vs interleaved sets.  sell_fits: whether G row groups of this lane
// layout fit in one wavefront.
bool sell_fits(int C, int elem_bytes, int G, bool wide);
template <typename T, typename TV>
hipError_t launch_sell(hipStream_t st, int C, int G, int64_t n, const int64_t* off, const int32_t* wid,
                       const int32_t* ci, const TV* va, const T* X, T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta,
                       OuterDiag sigma, int S, int m, int vs, bool wide = false, const int* gate = nullptr);
template <typename T>
hipError_t launch_dot(hipStream_t st, int C, int64_t n, const T* X, const T* Y, double* partial, int nb,
                      double* out);

// x += alpha p (every column; alpha = 0 on frozen ones), then p = z + beta p on active columns;
// gated: nothing runs when every alpha is zero
hipError_t launch_pcg_pupdate(hipStream_t st, int C, int64_t n, double* x, double* p, const double* z,
                              const double* alpha, const double* beta, const int* active, bool gated = false);

hipError_t launch_qs_forward(hipStream_t st, int S, int64_t n_b, int m, int C, int64_t n, const int64_t* img,
                             const double* b, double* out);
// p != nullptr: transforms xh + alpha p (alpha per column), the x step of an
// iteration that ended the solve before its p update
hipError_t launch_qs_backward(hipStream_t st, int S, int64_t n_b, int m, int C, int64_t n, const int64_t* img,
                              const double* xh, double* x, const double* p = nullptr, const double* alpha = nullptr);
// out[j] = ||b_j||^2 for the m columns of an n x m column-major array (partial: nb * m scratch)
hipError_t launch_colnorm2(hipStream_t st, int64_t n, int m, const double* b, double* partial, int nb,
                           double* out);
hipError_t launch_thresholds(hipStream_t st, int C, int S, int m, double tol, const double* bn2, double* thr);

// out = Minv y (dense FP64 coarsest solve, split over k; part: dense_splits(C, nL, sizeof(T)) * nL * C doubles)
int dense_splits(int C, int64_t nL, int elem_bytes);
template <typename T>
hipError_t launch_dense(hipStream_t st, int C, int64_t nL, const double* Minv, const T* y, T* out, double* part,
                        const int* gate = nullptr);
// Per-subsystem coarsest solves: columns a*m .. a*m + m - 1 times the
// inverse Minv + a*nL*ld (S inverses, rows of ld = dense_sets_ld(nL,
// sizeof(TM)) entries, the ones past nL zero; TM = double or float); columns
// >= S*m of out are zero.  yp: scratch of S * ld * MP values, MP = m rounded
// up to a power of two (at most 2 * (nL + 4) * C).  R: rows per wavefront
// (1, 2, 4 or 8; capped at dense_sets_rows_max(m)).
int dense_sets_rows_max(int m);
int64_t dense_sets_ld(int64_t nL, int minv_bytes);
template <typename T, typename TM>
hipError_t launch_dense_sets(hipStream_t st, int C, int S, int m, int64_t nL, const TM* Minv, const T* y, T* out,
                             T* yp, int R, const int* gate = nullptr);
template <typename T>
hipError_t launch_fill(hipStream_t st, int64_t len, T* p, T v);
template <typename TO, typename TI>
hipError_t launch_cast(hipStream_t st, int64_t len, const TI* a, TO* b);

// Device scratch of the allocation-free solve: a file-scope device array of
// kScratchBytes per GPU.  scratch_init looks up its address on the current
// device (once per device); scratch_address returns it (nullptr before).
constexpr size_t kScratchBytes = size_t(128) << 20;
hipError_t scratch_init();
void* scratch_address(int device);

// flags[0..1] to fine-grained host memory pub (device-visible pointer), then pub[2] = seq
hipError_t launch_publish_flags(hipStream_t st, const int* flags, int* pub, int seq);
// flags of every system of a batch into one array (2 ints per system)
hipError_t launch_gather_flags(hipStream_t st, int nsys, int* const* ptrs, int* out);

// dL/dkappa per base cell from face products (see msp_fv_kappa_grad)
hipError_t launch_kappa_grad(hipStream_t st, int64_t n_b, int S, int64_t n, int m, const int64_t* cfp,
                            const int32_t* cfi, const int64_t* img, const int64_t* ca, const int64_t* cb,
                            const int8_t* kind, const int8_t* axis, const double* area, const double* da,
                            const double* db, const double* kap, const double* lam, const double* p, double* grad);

// column-wise: X[:, c] *= f[c]; Y[:, c] -= h[c] X[:, c]  (len = rows * C)
template <typename T>
hipError_t launch_scale_cols(hipStream_t st, int64_t len, int C, T* X, const double* f);
hipError_t launch_axpy_cols(hipStream_t st, int64_t len, int C, double* Y, const double* X, const double* h);

// Low-rank corrections; U is n x (S*k): U[i, a*k+t].
// combine: U[i, a*k+t] = sum_j V_j[i, a] cm[(a*K + j)*k + t]  (V: K blocks of n x C)
template <typename TU>
hipError_t launch_lrc_combine(hipStream_t st, int64_t n, int S, int k, int K, int C, const double* V,
                              const double* cm, TU* U);
// apply: Z[:, a*m+j] += U_a diag(coef_a) U_a^T R[:, a*m+j]  (partial: nb * S*k*m, W: S*k*m scratch)
template <typename TU>
hipError_t launch_lrc_apply(hipStream_t st, int64_t n, int S, int k, int m, int C, const TU* U, const double* R,
                            double* Z, const double* coef, double* partial, int nb, double* W);

}  // namespace msp
