// Launchers of the numeric re-setup kernels (refresh.hip).  Matrices are CSR
// with int32 row pointers and columns; every launch is asynchronous on `st`;
// `err` (device int) collects pattern misses of the interpolation (1) and
// non-positive FSAI pivots (2).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace msp {

// out[i * stride + offset] = src[i] >= 0 ? in[src[i]] : 0, i < n
hipError_t launch_gather(hipStream_t st, int64_t n, const int64_t* src, const double* in, double* out, int stride = 1,
                         int offset = 0);
// out[i * ostride + ooff] = in[i * istride + ioff], i < n
hipError_t launch_strided_copy(hipStream_t st, int64_t n, const double* in, int istride, int ioff, double* out,
                               int ostride, int ooff);
// sigma (nb x S) of eq. (2.14) from the outer couplings h_j(i) = val[src[i*(S-1) + j-1]] (-1: none)
hipError_t launch_outer_sigma(hipStream_t st, int64_t nb, int S, const int64_t* src, const double* val,
                              double* sigma);
// v[diag[q]] += sigma[base[q] * S + a], q < nq
hipError_t launch_add_sigma(hipStream_t st, int64_t nq, const int64_t* diag, const int64_t* base,
                            const double* sigma, int S, int a, double* v);
// one Jacobi step of the interpolation on the F rows (prp == nullptr: the first step, -D^{-1} A_FC);
// afc and hasf are scratch of W's size
hipError_t launch_interp_step(hipStream_t st, int64_t nf, const int32_t* fidx, const int32_t* arp,
                              const int32_t* aci, const double* av, const int8_t* cf, const int32_t* cnum,
                              const int32_t* fnum, const int32_t* prp, const int32_t* pci, const double* pv,
                              const int32_t* wrp, const int32_t* wci, double* wv, double* afc, int8_t* hasf,
                              int* err);
// P values: unit rows for C points, the kept weights (pmap into wv) rescaled for F points
hipError_t launch_interp_finish(hipStream_t st, int64_t n, const int8_t* cf, const int32_t* arp, const int32_t* aci,
                                const double* av, const double* wv, const int32_t* prp, const int32_t* pmap,
                                double* pv);
// static FSAI rows on G's pattern; work + woff[i] holds k_i^2 + k_i doubles for row i
hipError_t launch_fsai(hipStream_t st, int64_t n, const int32_t* arp, const int32_t* aci, const double* av,
                       const int32_t* grp, const int32_t* gci, double* gv, const int64_t* woff, double* work,
                       int* err);
// C = A B on C's kept pattern (nr rows, nnz entries), which holds every
// product term (a symbolic product of the kept patterns)
hipError_t launch_spgemm_masked(hipStream_t st, int64_t nr, int64_t nnz, const int32_t* arp, const int32_t* aci,
                                const double* av, const int32_t* brp, const int32_t* bci, const double* bv,
                                const int32_t* crp, const int32_t* cci, double* cv);
hipError_t launch_scale(hipStream_t st, int64_t n, double* v, double s);
// y = M x (n rows, nnz entries: rows of 32 or more entries on average take a wavefront each)
hipError_t launch_spmv(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci, const double* v,
                       const double* x, double* y, int64_t nnz);
// values of a sliced-ELL form (slots x vs sets; FP32 if out32) from CSR values, pos: slot -> entry (-1: padding)
hipError_t launch_sell_values(hipStream_t st, int64_t slots, int vs, const int64_t* pos, const double* v,
                              double* out64, float* out32);
// out[0] = v.w, out[1] = w.w (nb block partials in part, 2 * nb doubles)
hipError_t launch_power_dots(hipStream_t st, int64_t n, const double* v, const double* w, double* part, int nb,
                             double* out);
// v = w / sqrt(dots[1])
hipError_t launch_normalise(hipStream_t st, int64_t n, const double* w, const double* dots, double* v);
// X (S blocks of n x n, row-major) = inverse of the S value sets of the SPD CSR matrix (set a at v[k*S + a]),
// Gauss-Jordan without pivoting; rowk, colk: S * n doubles of scratch
hipError_t launch_dense_inverse(hipStream_t st, int64_t n, int S, const int32_t* rp, const int32_t* ci,
                                const double* v, double* X, double* rowk, double* colk);

// out (S * n rows of ld floats) = X (S * n rows of n doubles), padding zero
hipError_t launch_dense_to_f32(hipStream_t st, int S, int64_t n, int64_t ld, const double* X, float* out);

// energy minimisation of an interpolation P (n rows; cf: C rows are unit rows, left alone):
// out = sign * (v - row mean of v) on F rows, 0 on C rows
hipError_t launch_emin_project(hipStream_t st, int64_t n, const int32_t* rp, const int8_t* cf, const double* v,
                               double sign, double* out);
// dinv[k] = 1 / a_ii for the entries k of row i of P
hipError_t launch_emin_dinv(hipStream_t st, int64_t n, const int32_t* arp, const int32_t* aci, const double* av,
                            const int32_t* prp, double* dinv);
// w += alpha p, r -= alpha q, z = dinv r (m entries)
hipError_t launch_emin_step(hipStream_t st, int64_t m, double alpha, const double* p, const double* q,
                            const double* dinv, double* w, double* r, double* z);
// p = z + beta p
hipError_t launch_emin_dir(hipStream_t st, int64_t m, double beta, const double* z, double* p);
// out = a * b elementwise
hipError_t launch_mul(hipStream_t st, int64_t m, const double* a, const double* b, double* out);

// Split of the reduction level for new values (Alg. 2): strength mask of every entry of A (smask) and its
// symmetric closure (tmask; tmap: entry (i, j) -> entry (j, i))
hipError_t launch_split_strength(hipStream_t st, int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                                 const double* v, double theta, const int64_t* tmap, int8_t* smask, int8_t* tmask);
// one round of the distance-d (d <= 3) maximal independent set under the priorities (lam, then pri; lam may
// be nullptr) over the candidates (state: 0 undecided, 1 in, 2 out, 3 not a candidate); *left += undecided
// candidates after the round
hipError_t launch_mis_round(hipStream_t st, int64_t n, int d, const int32_t* rp, const int32_t* ci,
                            const int8_t* tmask, const int32_t* lam, const uint64_t* pri, int8_t* state, int* left);
// lam[i] += number of rows whose strong set (smask) holds i
hipError_t launch_strong_dependants(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci,
                                   const int8_t* smask, int32_t* lam);
// *count += points whose C/F decision (in or not a candidate: C) differs from cf
hipError_t launch_split_diff(hipStream_t st, int64_t n, const int8_t* state, const int8_t* cf,
                             unsigned long long* count);

// finite-volume values on the device: T per face, the diagonal per base cell,
// then val[p] = slot[p] >= 0 ? -T[slot[p]] : diag[-slot[p] - 1]
hipError_t launch_fv_values(hipStream_t st, int64_t nf, int64_t nb, int64_t nnz, const int64_t* ca, const int64_t* cb,
                            const int8_t* kind, const double* area, const double* da, const double* db,
                            const int64_t* cfp, const int32_t* cfi, const int32_t* slot, const double* kap, double* T,
                            double* diag, double* val);

}  // namespace msp
