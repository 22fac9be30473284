// Launchers of the fused PCG kernels (pcg.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "kernels.hpp"

namespace msp {

constexpr int kPcgMaxBlocks = 2048;   // largest grid of the dot-producing kernels (grid-stride over row tiles)

// Grids of the dot-producing kernels over n rows: the row tiles, capped at
// kPcgMaxBlocks and at the blocks of that kernel the current device holds at
// once.  The partial arrays they fill have nb rows; the finisher that reads
// them takes the same nb.  update_dots_grid sizes the updating variant (the
// initial, non-updating one uses fewer registers and fits the same grid).
hipError_t op_dot_grid(int C, bool sell, int64_t n, int* nb);
template <typename TU>
hipError_t update_dots_grid(int C, int k, int64_t n, int* nb);
template <typename TS, typename TU>
hipError_t zfinish_grid(int C, bool lrc, bool flex, int64_t n, int* nb);

// sl.ci != nullptr: the operator in its sliced-ELL form (one group per row)
hipError_t launch_op_dot(hipStream_t st, int C, int nb, int64_t n, const int32_t* rp, const int32_t* ci,
                         const double* va, SellRef sl, OuterDiag sigma, int S, int m, const double* p, double* q,
                         double* partial, const int* gate = nullptr);
hipError_t launch_fin_alpha(hipStream_t st, int C, int nb, const double* partial, const int* active,
                            const double* rho, double* alpha, double* pq, int* flags);
// upd: r -= alpha q (x is updated by launch_pcg_pupdate, or by the back transform after the last iteration)
template <typename TU>
hipError_t launch_update_dots(hipStream_t st, int C, int nb, bool upd, int k, int64_t n, double* r, const double* q,
                              const double* alpha, const TU* U, int S, int m, double* prr, double* plrc, float* y32,
                              Bf16* y16, const int* gate = nullptr);
hipError_t launch_fin_check(hipStream_t st, int C, int nb, bool init, int O, int m, const double* prr,
                            const double* plrc, const double* thr, const double* coef, int* active, int* iters,
                            int* flags, double* rnorm, double* W);
// z == nullptr: z is not stored.  z2 != nullptr: z also written there (the
// first search direction p = z).
// q != nullptr (flexible beta): partial_qz also receives the partials of <q, z>.
template <typename TS, typename TU>
hipError_t launch_zfinish(hipStream_t st, int C, int nb, int64_t n, const TS* s, double* z, const double* r,
                          const TU* U, const double* W, int S, int k, int m, double* partial, double* z2 = nullptr,
                          const double* q = nullptr, double* partial_qz = nullptr, const int* gate = nullptr);
// The p update of the mixed modes, which store no z: x += alpha p, then
// p = z + beta p with z rebuilt from the V-cycle output s and U W (bit for bit
// the z of launch_zfinish with the same s, U, W).  Grid-stride; nb from
// pupdate_rebuild_grid.  S * k * m <= 1024 when U is given.
template <typename TS, typename TU>
hipError_t pupdate_rebuild_grid(int C, bool lrc, int64_t n, int* nb);
template <typename TS, typename TU>
hipError_t launch_pupdate_rebuild(hipStream_t st, int C, int nb, int64_t n, double* x, double* p, const TS* s,
                                  const TU* U, const double* W, int S, int k, int m, const double* alpha,
                                  const double* beta, const int* active, bool gated);
// flex (non-initial calls): beta = -<q,z>/<p,q> from partial_qz and pq
hipError_t launch_fin_beta(hipStream_t st, int C, int nb, bool init, bool flex, const double* partial,
                           const double* partial_qz, const int* active, const double* pq, double* rho, double* beta,
                           double* rz, const int* gate = nullptr);

}  // namespace msp
