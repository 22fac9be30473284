// Fused kernels of the per-column PCG (Alg. 1, decoupled solves) on n_b x C
// FP64 multivectors.  Every dot product is produced inside the kernel that
// writes one of its operands (per-block column partials), and a small
// finishing kernel with one block per output sums the partials in a fixed
// order and takes the per-column scalar step (alpha, convergence check,
// beta), so a PCG iteration is:
//   op_dot -> fin_alpha -> update_dots -> fin_check -> [V-cycle] ->
//   zfinish -> fin_beta -> pupdate.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "device.hpp"
#include "pcg.hpp"

namespace msp {

template <int C>
using DL = Lanes<double, C>;

// low-rank projections reduced per LDS pass in k_update_dots (LDS: 4 * 256 * VW doubles,
// small enough that registers, not LDS, bound the kernel's occupancy)
constexpr int kUpdTch = 4;


// q = (A_inn + diag-outer) p; partial[b, c] = this block's sum of p[:, c] q[:, c]
// (sigma.idx must be set: the operator always has the outer diagonal).
// SELL: A_inn in the sliced-ELL form of sell.hip with one group per row
// (sl.off, sl.wid, sl.ci, sl.va): the column indices and values of 8 entries
// are loaded together, then their 8 gathers, with no row-pointer load.
template <int C, bool SELL>
__global__ __launch_bounds__(kBlock) void k_op_dot(int64_t n, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci, const double* __restrict__ va,
                                                   SellRef sl, OuterDiag sigma, int S, int m,
                                                   const double* __restrict__ p, double* __restrict__ q,
                                                   double* __restrict__ partial, const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    constexpr int VW = DL<C>::VW, LPR = DL<C>::LPR, RPB = DL<C>::RPB;
    __shared__ double sm[kBlock * VW];
    const int slot = threadIdx.x / LPR, lane = threadIdx.x % LPR;
    const int64_t ntiles = (n + RPB - 1) / RPB;
    double dacc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) dacc[e] = 0.0;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t row = tile * RPB + slot;
        if (row >= n) continue;
        double acc[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] = 0.0;
        if constexpr (SELL) {
            const int64_t sidx = row / 64;
            const int w = sl.wid[sidx];
            const int64_t q0 = sl.off[sidx] + row % 64;
            for (int k0 = 0; k0 < w; k0 += 8) {
                int32_t cc[8];
                double aa[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool in = k0 + u < w;
                    cc[u] = in ? sl.ci[q0 + (int64_t)(k0 + u) * 64] : -1;
                    aa[u] = in ? sl.va[q0 + (int64_t)(k0 + u) * 64] : 0.0;
                }
                Pack<double, VW> xs[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (cc[u] >= 0) {
                        xs[u] = ld<double, VW>(p + (int64_t)cc[u] * C + lane * VW);
                    } else {
#pragma unroll
                        for (int e = 0; e < VW; ++e) xs[u].e[e] = 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int e = 0; e < VW; ++e) acc[e] += aa[u] * xs[u].e[e];
            }
        } else if constexpr (LPR >= 4) {
            row_accumulate_bcast<double, C, VW, LPR>(rp[row], rp[row + 1], ci, va, p, lane,
                                                     (int)(threadIdx.x % 64) - lane, acc);
        } else {
            row_accumulate<double, C, VW>(rp[row], rp[row + 1], 1, ci, va, p, lane, acc);
        }
        const Pack<double, VW> pr = ld<double, VW>(p + row * C + lane * VW);
        const int32_t sq = sigma.idx[row];   // interface row: its outer diagonal
        Pack<double, VW> out;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int a = (lane * VW + e) / m;
            if (sq >= 0 && a < S) acc[e] += sigma.val[(int64_t)sq * S + a] * pr.e[e];
            out.e[e] = acc[e];
            dacc[e] += pr.e[e] * acc[e];
        }
        st<double, VW>(q + row * C + lane * VW, out);
    }
    block_column_sums<C, VW>(dacc, sm, partial + (int64_t)blockIdx.x * C);
}

// alpha[c] = rho[c] / <p,q>[c] on active columns (breakdown flag otherwise);
// resets the active-column counter flags[1] for this iteration's check.
__global__ __launch_bounds__(kBlock) void k_fin_alpha(int nb, int C, const double* __restrict__ partial,
                                                      const int* __restrict__ active, const double* __restrict__ rho,
                                                      double* __restrict__ alpha, double* __restrict__ pq, int* flags) {
    __shared__ double sm[kBlock];
    const int c = blockIdx.x;
    const double s = block_sum_partials(nb, C, c, partial, sm);
    if (threadIdx.x == 0) {
        pq[c] = s;
        double a = 0.0;
        if (active[c]) {
            if (!(s > 0.0) || !isfinite(s) || !isfinite(rho[c])) atomicOr(&flags[0], 1);
            else a = rho[c] / s;
        }
        alpha[c] = a;
        if (c == 0) flags[1] = 0;
    }
}

// UPD: r -= alpha q (the matching x += alpha p is applied by the p update,
// which reads p anyway).  Then per-block partials of <r,r> (partial_rr) and
// of the low-rank projections U_a^T r_a when KMAX > 0:
// partial_lrc[b, (a*k + t)*m + j] = sum_rows U[i, a*k+t] r[i, a*m+j].
template <int C, bool UPD, int KMAX, typename TU>
__global__ __launch_bounds__(kBlock) void k_update_dots(int64_t n, double* __restrict__ r,
                                                        const double* __restrict__ q,
                                                        const double* __restrict__ alpha, const TU* __restrict__ U,
                                                        int S, int k, int m, double* __restrict__ partial_rr,
                                                        double* __restrict__ partial_lrc, float* __restrict__ y32,
                                                        Bf16* __restrict__ y16, const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    constexpr int VW = DL<C>::VW, LPR = DL<C>::LPR, RPB = DL<C>::RPB;
    constexpr int KA = KMAX > 0 ? KMAX : 1;
    __shared__ double sm[kBlock * VW];
    const int slot = threadIdx.x / LPR, lane = threadIdx.x % LPR;
    const int64_t ntiles = (n + RPB - 1) / RPB;
    // each thread's share of the projections (about a dozen rows) is summed in
    // FP32 when U is bfloat16 (it frees the registers that bound the occupancy);
    // block and grid sums are FP64
    using TA = typename std::conditional<std::is_same<TU, Bf16>::value, float, double>::type;
    double a_rr[VW];
    TA a_l[VW][KA];
    double al[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        a_rr[e] = 0.0;
        al[e] = UPD ? alpha[lane * VW + e] : 0.0;
#pragma unroll
        for (int t = 0; t < KA; ++t) a_l[e][t] = TA(0);
    }
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t row = tile * RPB + slot;
        if (row >= n) continue;
        const int64_t o = row * C + lane * VW;
        Pack<double, VW> rv = ld<double, VW>(r + o);
        if (UPD) {
            const Pack<double, VW> qv = ld<double, VW>(q + o);
#pragma unroll
            for (int e = 0; e < VW; ++e) rv.e[e] -= al[e] * qv.e[e];
            st<double, VW>(r + o, rv);
        }
        if (y32) {   // FP32 copy of r: the V-cycle input of the mixed mode
            Pack<float, VW> yv;
#pragma unroll
            for (int e = 0; e < VW; ++e) yv.e[e] = (float)rv.e[e];
            st<float, VW>(y32 + o, yv);
        }
        if (y16) {   // bfloat16 copy of r (V-cycle multivectors in bfloat16)
            Pack<Bf16, VW> yv;
#pragma unroll
            for (int e = 0; e < VW; ++e) yv.e[e] = from_double<Bf16>(rv.e[e]);
            st<Bf16, VW>(y16 + o, yv);
        }
#pragma unroll
        for (int e = 0; e < VW; ++e) a_rr[e] += rv.e[e] * rv.e[e];
        if (KMAX > 0) {
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const int col = lane * VW + e;
                const int a = col / m;
                if (a < S) {
                    const TU* u = U + row * (S * k) + a * k;
                    if ((k & 3) == 0) {
#pragma unroll
                        for (int t = 0; t < KA; t += 4)
                            if (t < k) {
                                const Pack<TU, 4> u4 = ld<TU, 4>(u + t);
#pragma unroll
                                for (int q = 0; q < 4 && t + q < KA; ++q)
                                    a_l[e][t + q] += (TA)to_acc(u4.e[q]) * (TA)rv.e[e];
                            }
                    } else {
#pragma unroll
                        for (int t = 0; t < KA; ++t)
                            if (t < k) a_l[e][t] += (TA)to_acc(u[t]) * (TA)rv.e[e];
                    }
                }
            }
        }
    }
    block_column_sums<C, VW>(a_rr, sm, partial_rr + (int64_t)blockIdx.x * C);
    if (KMAX > 0) {
        // kUpdTch projections per pass: slm[(tt * kBlock + thread) * VW + e] for t = t0 + tt,
        // then one thread per output (column, t) sums the RPB row slots in a fixed order
        extern __shared__ double slm[];
        const int O = S * k * m;
#pragma unroll
        for (int t0 = 0; t0 < KA; t0 += kUpdTch) {
            if (t0 >= k) break;
#pragma unroll
            for (int tt = 0; tt < kUpdTch && t0 + tt < KA; ++tt) {
#pragma unroll
                for (int e = 0; e < VW; ++e) slm[(tt * kBlock + threadIdx.x) * VW + e] = (double)a_l[e][t0 + tt];
            }
            __syncthreads();
            const int nt = k - t0 < kUpdTch ? k - t0 : kUpdTch;
            for (int q = threadIdx.x; q < S * m * nt; q += kBlock) {
                const int col = q % (S * m), tt = q / (S * m);
                double v = 0.0;
                for (int r = 0; r < RPB; ++r) v += slm[tt * kBlock * VW + r * C + col];
                const int a = col / m, j = col % m;
                partial_lrc[(int64_t)blockIdx.x * O + (a * k + t0 + tt) * m + j] = v;
            }
            __syncthreads();
        }
    }
}

// Blocks [0, C): <r,r> -> convergence check (INIT: set the active flags);
// the next S*k*m blocks when LRC: W[o] = coef[o / m] * U^T r.
__global__ __launch_bounds__(kBlock) void k_fin_check(int nb, int C, int init, int O, int m,
                                                      const double* __restrict__ partial_rr,
                                                      const double* __restrict__ partial_lrc,
                                                      const double* __restrict__ thr, const double* __restrict__ coef,
                                                      int* active, int* iters, int* flags, double* rnorm, double* W) {
    __shared__ double sm[kBlock];
    int b = blockIdx.x;
    if (b < C) {
        const double s = block_sum_partials(nb, C, b, partial_rr, sm);
        if (threadIdx.x == 0) {
            const double nr = sqrt(s);
            if (init) {
                rnorm[b] = nr;
                iters[b] = 0;
                if (!isfinite(nr) || !(thr[b] >= 0.0)) atomicOr(&flags[0], 1);   // non-finite right-hand side
                const int a = nr > thr[b] ? 1 : 0;
                active[b] = a;
                if (a) atomicAdd(&flags[1], 1);
            } else if (active[b]) {
                iters[b] += 1;
                rnorm[b] = nr;
                if (!isfinite(nr)) atomicOr(&flags[0], 1);
                if (nr > thr[b]) atomicAdd(&flags[1], 1);
                else active[b] = 0;
            }
        }
        return;
    }
    b -= C;
    if (b < O) {
        const double s = block_sum_partials(nb, O, b, partial_lrc, sm);
        if (threadIdx.x == 0) W[b] = coef[b / m] * s;
    }
}

// z = s (cast to FP64; s may alias z) + sum_t U[i, a*k+t] W[(a*k+t)*m + j]
// (the expansion of the low-rank correction); partial[b, c] = sum r z and,
// when FLEX, partial_qz[b, c] = sum q z (q = A p of this iteration: the
// numerator of the flexible beta).
// z of one row and lane: the V-cycle output s plus the low-rank correction
// U_a W_a of the lane's subsystems (wl: W staged in LDS).  The z-finish kernel
// and the rebuilding p update both form z through this function, so the two
// agree bit for bit.
template <int VW, typename TS, bool LRC, typename TU>
__device__ __forceinline__ Pack<double, VW> z_lane(int64_t row, int64_t o, int lane, const TS* s,
                                                   const TU* __restrict__ U, const double* wl, int S, int k, int m) {
    Pack<double, VW> zv;
    const Pack<TS, VW> sv = ld<TS, VW>(s + o);
#pragma unroll
    for (int e = 0; e < VW; ++e) zv.e[e] = (double)to_acc(sv.e[e]);
    if (LRC) {
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const int col = lane * VW + e;
            const int a = col / m, j = col % m;
            if (a < S) {
                const TU* u = U + row * (S * k) + a * k;
                const double* w = wl + (a * k) * m + j;
                double t2 = 0.0;
                int t = 0;
                for (; (k & 3) == 0 && t + 4 <= k; t += 4) {   // aligned 4-wide loads when k % 4 == 0
                    const Pack<TU, 4> u4 = ld<TU, 4>(u + t);
                    t2 += (double)to_acc(u4.e[0]) * w[t * m];
                    t2 += (double)to_acc(u4.e[1]) * w[(t + 1) * m];
                    t2 += (double)to_acc(u4.e[2]) * w[(t + 2) * m];
                    t2 += (double)to_acc(u4.e[3]) * w[(t + 3) * m];
                }
                for (; t < k; ++t) t2 += (double)to_acc(u[t]) * w[t * m];
                zv.e[e] += t2;
            }
        }
    }
    return zv;
}

// z == nullptr: z is not stored (the mixed modes, whose p update rebuilds it
// with k_pupdate_rebuild).  z2 != nullptr: z is written there (the first
// search direction).
template <int C, typename TS, bool LRC, typename TU, bool FLEX>
__global__ __launch_bounds__(kBlock) void k_zfinish(int64_t n, const TS* s, double* z, const double* __restrict__ r,
                                                    const TU* __restrict__ U, const double* __restrict__ W, int S,
                                                    int k, int m, double* __restrict__ partial,
                                                    double* __restrict__ z2, const double* __restrict__ q,
                                                    double* __restrict__ partial_qz, const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    constexpr int VW = DL<C>::VW, LPR = DL<C>::LPR, RPB = DL<C>::RPB;
    __shared__ double sm[kBlock * VW];
    __shared__ double wl[LRC ? 64 * 16 : 1];
    const int slot = threadIdx.x / LPR, lane = threadIdx.x % LPR;
    const int64_t ntiles = (n + RPB - 1) / RPB;
    if (LRC) {
        for (int o = threadIdx.x; o < S * k * m; o += kBlock) wl[o] = W[o];
        __syncthreads();
    }
    double acc[VW], aqz[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = aqz[e] = 0.0;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t row = tile * RPB + slot;
        if (row >= n) continue;
        const int64_t o = row * C + lane * VW;
        const Pack<double, VW> zv = z_lane<VW, TS, LRC, TU>(row, o, lane, s, U, wl, S, k, m);
        if (z) st<double, VW>(z + o, zv);
        if (z2) st<double, VW>(z2 + o, zv);
        const Pack<double, VW> rv = ld<double, VW>(r + o);
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] += rv.e[e] * zv.e[e];
        if (FLEX) {
            const Pack<double, VW> qv = ld<double, VW>(q + o);
#pragma unroll
            for (int e = 0; e < VW; ++e) aqz[e] += qv.e[e] * zv.e[e];
        }
    }
    block_column_sums<C, VW>(acc, sm, partial + (int64_t)blockIdx.x * C);
    if (FLEX) block_column_sums<C, VW>(aqz, sm, partial_qz + (int64_t)blockIdx.x * C);
}

// x += alpha p (this iteration's x step; alpha = 0 on frozen columns), then
// p = z + beta p on active columns, with z rebuilt from the V-cycle output s
// and U W exactly as the z-finish kernel formed it (the mixed modes store no
// z: s and U are read instead of the FP64 z).  Grid-stride over row tiles,
// W staged in LDS once per block.
template <int C, typename TS, bool LRC, typename TU>
__global__ __launch_bounds__(kBlock) void k_pupdate_rebuild(int64_t n, double* __restrict__ x, double* __restrict__ p,
                                                            const TS* __restrict__ s, const TU* __restrict__ U,
                                                            const double* __restrict__ W, int S, int k, int m,
                                                            const double* __restrict__ alpha,
                                                            const double* __restrict__ beta,
                                                            const int* __restrict__ active, int gated) {
    if (alpha_gate_closed(alpha, gated != 0)) return;
    constexpr int VW = DL<C>::VW, LPR = DL<C>::LPR, RPB = DL<C>::RPB;
    __shared__ double wl[LRC ? 64 * 16 : 1];
    const int slot = threadIdx.x / LPR, lane = threadIdx.x % LPR;
    const int64_t ntiles = (n + RPB - 1) / RPB;
    if (LRC) {
        for (int o = threadIdx.x; o < S * k * m; o += kBlock) wl[o] = W[o];
        __syncthreads();
    }
    double al[VW], be[VW];
    bool on[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        const int c = lane * VW + e;
        al[e] = alpha[c];
        be[e] = beta[c];
        on[e] = active[c] != 0;
    }
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t row = tile * RPB + slot;
        if (row >= n) continue;
        const int64_t o = row * C + lane * VW;
        Pack<double, VW> pv = ld<double, VW>(p + o);
        Pack<double, VW> xv = ld<double, VW>(x + o);
        const Pack<double, VW> zv = z_lane<VW, TS, LRC, TU>(row, o, lane, s, U, wl, S, k, m);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            xv.e[e] += al[e] * pv.e[e];
            if (on[e]) pv.e[e] = zv.e[e] + be[e] * pv.e[e];
        }
        st<double, VW>(x + o, xv);
        st<double, VW>(p + o, pv);
    }
}

// beta and rho = <r,z> on active columns; INIT: rho = <r,z> for every
// column.  Standard beta: <r,z>/rho.  Flexible (Notay's flexible CG with one
// kept direction): beta = -<z, A p>/<p, A p>, which keeps the new direction
// A-orthogonal to the last one when the preconditioner varies between
// iterations (the reduced-precision V-cycle).  Block c < C sums <r,z> and
// sets rho; when FLEX, block C + c sums <q,z> (q = A p) and sets beta from it
// and pq alone, so the two blocks of a column share no data.
__global__ __launch_bounds__(kBlock) void k_fin_beta(int nb, int C, int init, int flex,
                                                     const double* __restrict__ partial,
                                                     const double* __restrict__ partial_qz,
                                                     const int* __restrict__ active, const double* __restrict__ pq,
                                                     double* rho, double* beta, double* rz,
                                                     const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    __shared__ double sm[kBlock];
    const bool qz_block = (int)blockIdx.x >= C;
    const int c = qz_block ? blockIdx.x - C : blockIdx.x;
    const double s = block_sum_partials(nb, C, c, qz_block ? partial_qz : partial, sm);
    if (threadIdx.x != 0) return;
    if (qz_block) {   // flexible beta (non-initial calls only)
        beta[c] = active[c] ? -s / pq[c] : 0.0;
        return;
    }
    rz[c] = s;
    if (init) {
        rho[c] = s;
        beta[c] = 0.0;
    } else if (active[c]) {
        if (!flex) beta[c] = s / rho[c];
        rho[c] = s;
    } else if (!flex) {
        beta[c] = 0.0;
    }
}

// ------------------------------------------------------------------ launchers

#define MSP_DISPATCH_C(C, ...)                                   \
    switch (C) {                                                 \
        case 1: { constexpr int CC = 1; __VA_ARGS__; } break;    \
        case 2: { constexpr int CC = 2; __VA_ARGS__; } break;    \
        case 4: { constexpr int CC = 4; __VA_ARGS__; } break;    \
        case 8: { constexpr int CC = 8; __VA_ARGS__; } break;    \
        case 16: { constexpr int CC = 16; __VA_ARGS__; } break;  \
        case 32: { constexpr int CC = 32; __VA_ARGS__; } break;  \
        case 64: { constexpr int CC = 64; __VA_ARGS__; } break;  \
        default: return hipErrorInvalidValue;                    \
    }

// Blocks for a grid-stride kernel over n rows: its row tiles, at most
// kPcgMaxBlocks, and at most the blocks of this kernel that the device holds
// at once (its occupancy on one compute unit times the compute units), so
// that no block waits for a slot while the others run.
template <int C, typename K>
static hipError_t resident_grid(K kernel, size_t lds, int64_t n, int* nb) {
    const int64_t tiles = (n + DL<C>::RPB - 1) / DL<C>::RPB;
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(kernel), kBlock, lds);
    if (e != hipSuccess) return e;
    int64_t cap = kPcgMaxBlocks;
    if (per > 0 && cus > 0 && (int64_t)per * cus < cap) cap = (int64_t)per * cus;
    *nb = (int)(tiles < cap ? (tiles > 0 ? tiles : 1) : cap);
    return hipSuccess;
}

hipError_t op_dot_grid(int C, bool sell, int64_t n, int* nb) {
    MSP_DISPATCH_C(C, {
        return sell ? resident_grid<CC>(k_op_dot<CC, true>, 0, n, nb) : resident_grid<CC>(k_op_dot<CC, false>, 0, n, nb);
    });
    return hipErrorInvalidValue;
}

template <typename TU>
hipError_t update_dots_grid(int C, int k, int64_t n, int* nb) {
    if (k > 16) return hipErrorInvalidValue;
    MSP_DISPATCH_C(C, {
        constexpr size_t lds = sizeof(double) * kUpdTch * kBlock * DL<CC>::VW;
        if (k > 8) return resident_grid<CC>(k_update_dots<CC, true, 16, TU>, lds, n, nb);
        if (k > 0) return resident_grid<CC>(k_update_dots<CC, true, 8, TU>, lds, n, nb);
        return resident_grid<CC>(k_update_dots<CC, true, 0, TU>, 0, n, nb);
    });
    return hipErrorInvalidValue;
}
template hipError_t update_dots_grid<float>(int, int, int64_t, int*);
template hipError_t update_dots_grid<double>(int, int, int64_t, int*);
template hipError_t update_dots_grid<Bf16>(int, int, int64_t, int*);

template <typename TS, typename TU>
hipError_t zfinish_grid(int C, bool lrc, bool flex, int64_t n, int* nb) {
    MSP_DISPATCH_C(C, {
        if (flex)
            return lrc ? resident_grid<CC>(k_zfinish<CC, TS, true, TU, true>, 0, n, nb)
                       : resident_grid<CC>(k_zfinish<CC, TS, false, TU, true>, 0, n, nb);
        return lrc ? resident_grid<CC>(k_zfinish<CC, TS, true, TU, false>, 0, n, nb)
                   : resident_grid<CC>(k_zfinish<CC, TS, false, TU, false>, 0, n, nb);
    });
    return hipErrorInvalidValue;
}
template hipError_t zfinish_grid<float, float>(int, bool, bool, int64_t, int*);
template hipError_t zfinish_grid<double, double>(int, bool, bool, int64_t, int*);
template hipError_t zfinish_grid<double, float>(int, bool, bool, int64_t, int*);
template hipError_t zfinish_grid<float, double>(int, bool, bool, int64_t, int*);
template hipError_t zfinish_grid<Bf16, float>(int, bool, bool, int64_t, int*);
template hipError_t zfinish_grid<Bf16, double>(int, bool, bool, int64_t, int*);
template hipError_t zfinish_grid<Bf16, Bf16>(int, bool, bool, int64_t, int*);

template <typename TS, typename TU>
hipError_t pupdate_rebuild_grid(int C, bool lrc, int64_t n, int* nb) {
    MSP_DISPATCH_C(C, {
        return lrc ? resident_grid<CC>(k_pupdate_rebuild<CC, TS, true, TU>, 0, n, nb)
                   : resident_grid<CC>(k_pupdate_rebuild<CC, TS, false, TU>, 0, n, nb);
    });
    return hipErrorInvalidValue;
}

template <typename TS, typename TU>
hipError_t launch_pupdate_rebuild(hipStream_t st, int C, int nb, int64_t n, double* x, double* p, const TS* s,
                                  const TU* U, const double* W, int S, int k, int m, const double* alpha,
                                  const double* beta, const int* active, bool gated) {
    if (U && k > 0 && S * k * m > 64 * 16) return hipErrorInvalidValue;
    MSP_DISPATCH_C(C, {
        if (U && k > 0)
            hipLaunchKernelGGL((k_pupdate_rebuild<CC, TS, true, TU>), dim3(nb), dim3(kBlock), 0, st, n, x, p, s, U, W,
                               S, k, m, alpha, beta, active, gated ? 1 : 0);
        else
            hipLaunchKernelGGL((k_pupdate_rebuild<CC, TS, false, TU>), dim3(nb), dim3(kBlock), 0, st, n, x, p, s, U, W,
                               S, k, m, alpha, beta, active, gated ? 1 : 0);
    });
    return hipGetLastError();
}
#define MSP_PUPDATE_INST(TS, TU)                                                                                   \
    template hipError_t pupdate_rebuild_grid<TS, TU>(int, bool, int64_t, int*);                                     \
    template hipError_t launch_pupdate_rebuild<TS, TU>(hipStream_t, int, int, int64_t, double*, double*, const TS*, \
                                                       const TU*, const double*, int, int, int, const double*,      \
                                                       const double*, const int*, bool);
MSP_PUPDATE_INST(float, float)
MSP_PUPDATE_INST(float, double)
MSP_PUPDATE_INST(Bf16, float)
MSP_PUPDATE_INST(Bf16, double)
MSP_PUPDATE_INST(Bf16, Bf16)

hipError_t launch_op_dot(hipStream_t st, int C, int nb, int64_t n, const int32_t* rp, const int32_t* ci,
                         const double* va, SellRef sl, OuterDiag sigma, int S, int m, const double* p, double* q,
                         double* partial, const int* gate) {
    MSP_DISPATCH_C(C, {
        if (sl.ci)
            hipLaunchKernelGGL((k_op_dot<CC, true>), dim3(nb), dim3(kBlock), 0, st, n, rp, ci, va, sl, sigma, S, m, p,
                               q, partial, gate);
        else
            hipLaunchKernelGGL((k_op_dot<CC, false>), dim3(nb), dim3(kBlock), 0, st, n, rp, ci, va, sl, sigma, S, m, p,
                               q, partial, gate);
    });
    return hipGetLastError();
}

hipError_t launch_fin_alpha(hipStream_t st, int C, int nb, const double* partial, const int* active,
                            const double* rho, double* alpha, double* pq, int* flags) {
    hipLaunchKernelGGL(k_fin_alpha, dim3(C), dim3(kBlock), 0, st, nb, C, partial, active, rho, alpha, pq, flags);
    return hipGetLastError();
}

template <int CC, bool UPD, int KMAX, typename TU>
static void upd_launch(hipStream_t st, int nb, int64_t n, double* r, const double* q, const double* alpha,
                       const TU* U, int S, int k, int m, double* prr, double* plrc, float* y32, Bf16* y16,
                       const int* gate) {
    constexpr int VW = DL<CC>::VW;
    const size_t lds = KMAX > 0 ? sizeof(double) * kUpdTch * kBlock * VW : 0;   // projection partials per pass
    hipLaunchKernelGGL((k_update_dots<CC, UPD, KMAX, TU>), dim3(nb), dim3(kBlock), lds, st, n, r, q, alpha, U, S, k,
                       m, prr, plrc, y32, y16, gate);
}

template <typename TU>
hipError_t launch_update_dots(hipStream_t st, int C, int nb, bool upd, int k, int64_t n, double* r, const double* q,
                              const double* alpha, const TU* U, int S, int m, double* prr, double* plrc, float* y32,
                              Bf16* y16, const int* gate) {
    if (k > 16) return hipErrorInvalidValue;
    MSP_DISPATCH_C(C, {
        if (k > 8) {
            if (upd) upd_launch<CC, true, 16, TU>(st, nb, n, r, q, alpha, U, S, k, m, prr, plrc, y32, y16, gate);
            else upd_launch<CC, false, 16, TU>(st, nb, n, r, q, alpha, U, S, k, m, prr, plrc, y32, y16, gate);
        } else if (k > 0) {
            if (upd) upd_launch<CC, true, 8, TU>(st, nb, n, r, q, alpha, U, S, k, m, prr, plrc, y32, y16, gate);
            else upd_launch<CC, false, 8, TU>(st, nb, n, r, q, alpha, U, S, k, m, prr, plrc, y32, y16, gate);
        } else {
            if (upd) upd_launch<CC, true, 0, TU>(st, nb, n, r, q, alpha, U, S, k, m, prr, plrc, y32, y16, gate);
            else upd_launch<CC, false, 0, TU>(st, nb, n, r, q, alpha, U, S, k, m, prr, plrc, y32, y16, gate);
        }
    });
    return hipGetLastError();
}
template hipError_t launch_update_dots<float>(hipStream_t, int, int, bool, int, int64_t, double*, const double*,
                                              const double*, const float*, int, int, double*, double*, float*,
                                              Bf16*, const int*);
template hipError_t launch_update_dots<double>(hipStream_t, int, int, bool, int, int64_t, double*, const double*,
                                               const double*, const double*, int, int, double*, double*, float*,
                                               Bf16*, const int*);
template hipError_t launch_update_dots<Bf16>(hipStream_t, int, int, bool, int, int64_t, double*, const double*,
                                             const double*, const Bf16*, int, int, double*, double*, float*, Bf16*, const int*);

hipError_t launch_fin_check(hipStream_t st, int C, int nb, bool init, int O, int m, const double* prr,
                            const double* plrc, const double* thr, const double* coef, int* active, int* iters,
                            int* flags, double* rnorm, double* W) {
    const unsigned blocks = (unsigned)(C + O);
    hipLaunchKernelGGL(k_fin_check, dim3(blocks), dim3(kBlock), 0, st, nb, C, init ? 1 : 0, O, m, prr, plrc, thr,
                       coef, active, iters, flags, rnorm, W);
    return hipGetLastError();
}

template <int CC, typename TS, bool LRC, typename TU>
static void zfinish_launch(hipStream_t st, int nb, int64_t n, const TS* s, double* z, const double* r, const TU* U,
                           const double* W, int S, int k, int m, double* partial, double* z2, const double* q,
                           double* partial_qz, const int* gate) {
    if (q)
        hipLaunchKernelGGL((k_zfinish<CC, TS, LRC, TU, true>), dim3(nb), dim3(kBlock), 0, st, n, s, z, r, U, W, S, k,
                           m, partial, z2, q, partial_qz, gate);
    else
        hipLaunchKernelGGL((k_zfinish<CC, TS, LRC, TU, false>), dim3(nb), dim3(kBlock), 0, st, n, s, z, r, U, W, S, k,
                           m, partial, z2, q, partial_qz, gate);
}

template <typename TS, typename TU>
hipError_t launch_zfinish(hipStream_t st, int C, int nb, int64_t n, const TS* s, double* z, const double* r,
                          const TU* U, const double* W, int S, int k, int m, double* partial, double* z2,
                          const double* q, double* partial_qz, const int* gate) {
    if (q && !partial_qz) return hipErrorInvalidValue;
    MSP_DISPATCH_C(C, {
        if (U && k > 0) zfinish_launch<CC, TS, true, TU>(st, nb, n, s, z, r, U, W, S, k, m, partial, z2, q, partial_qz, gate);
        else zfinish_launch<CC, TS, false, TU>(st, nb, n, s, z, r, U, W, S, k, m, partial, z2, q, partial_qz, gate);
    });
    return hipGetLastError();
}
#define MSP_ZFINISH_INST(TS, TU)                                                                                  \
    template hipError_t launch_zfinish<TS, TU>(hipStream_t, int, int, int64_t, const TS*, double*, const double*,    \
                                               const TU*, const double*, int, int, int, double*, double*,           \
                                               const double*, double*, const int*);
MSP_ZFINISH_INST(float, float)
MSP_ZFINISH_INST(double, double)
MSP_ZFINISH_INST(double, float)
MSP_ZFINISH_INST(float, double)
MSP_ZFINISH_INST(Bf16, float)
MSP_ZFINISH_INST(Bf16, double)
MSP_ZFINISH_INST(Bf16, Bf16)

hipError_t launch_fin_beta(hipStream_t st, int C, int nb, bool init, bool flex, const double* partial,
                           const double* partial_qz, const int* active, const double* pq, double* rho, double* beta,
                           double* rz, const int* gate) {
    const bool fq = flex && !init;
    if (fq && (!partial_qz || !pq)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fin_beta, dim3(fq ? 2 * C : C), dim3(kBlock), 0, st, nb, C, init ? 1 : 0, fq ? 1 : 0, partial,
                       partial_qz, active, pq, rho, beta, rz, gate);
    return hipGetLastError();
}

}  // namespace msp
