// HIP kernels for gfx950 (CDNA4, wave64).
//
// Multivectors are n x C row-major (the C columns of one row are contiguous;
// C is the padded column count 2^s * m rounded up to a power of two).  A row
// is handled by LPR = C / VW lanes, each lane owning VW consecutive columns,
// so one wavefront covers 64 / LPR rows and every matrix entry (column index
// and value) is read once for all C columns (the SpMM of eq. (2.8)).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace msp {

// ------------------------------------------------------------------ SpMM
// Y = alpha * (A X + diag-outer(X)) + beta * Z, where the outer term adds
// sigma_a[row] * X[row, col], a = col / m (the per-subsystem outer diagonal of
// eq. (2.14), one value per subsystem, broadcast over its m columns; only
// rows listed in the compact OuterDiag carry it).
// Y may alias Z (each lane reads its own Z elements before writing them).
// With SETS the matrix holds vs interleaved value sets (entry k of set a at
// va[k * vs + a]) and column c is multiplied by set min(c / m, vs - 1): one
// pass applies a different operator of one sparsity pattern to every
// subsystem's columns.
// T is the storage type of the multivectors; arithmetic is in acc_t<T>.
// WIDE: 16-byte lanes (Lanes<T, C, true>; matrices with one value set).
template <typename T, typename TV, int C, bool SETS, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_spmm(int64_t n, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci,
                                                 const TV* __restrict__ va, const T* __restrict__ X,
                                                 T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta,
                                                 OuterDiag sigma, int S, int m, int vs, const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    using L = Lanes<T, C, WIDE>;
    using TC = acc_t<T>;
    constexpr int VW = L::VW;
    const int64_t row = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * L::RPB + threadIdx.x / L::LPR;
    const int lane = threadIdx.x % L::LPR;
    if (row >= n) return;
    TC acc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = TC(0);
    constexpr bool BC = L::LPR >= 4;   // broadcast row entries across the row's lanes
    const int base = (int)(threadIdx.x % 64) - lane;
    if constexpr (SETS) {
        int set[VW];
        const bool uniform = column_sets<VW>(lane, vs, m, set);
        if constexpr (BC) {   // all lanes of the row together (shuffles)
            row_accumulate_bcast_sets<T, C, VW, L::LPR, TV>(rp[row], rp[row + 1], ci, va, X, lane, base, acc, vs, set,
                                                            uniform);
        } else {
            if (uniform)
                row_accumulate<T, C, VW, TV, true>(rp[row], rp[row + 1], 1, ci, va + set[0], X, lane, acc, vs);
            else
                row_accumulate_sets<T, C, VW, TV>(rp[row], rp[row + 1], 1, ci, va, X, lane, acc, vs, set);
        }
    } else {
        if constexpr (BC)
            row_accumulate_bcast<T, C, VW, L::LPR, TV>(rp[row], rp[row + 1], ci, va, X, lane, base, acc);
        else
            row_accumulate<T, C, VW, TV>(rp[row], rp[row + 1], 1, ci, va, X, lane, acc);
    }
    if (sigma.idx) {
        const int32_t q = sigma.idx[row];
        if (q >= 0) {
            const Pack<T, VW> x = ld<T, VW>(X + row * C + lane * VW);
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const int a = (lane * VW + e) / m;
                if (a < S) acc[e] += (TC)sigma.val[(int64_t)q * S + a] * to_acc(x.e[e]);
            }
        }
    }
    Pack<T, VW> out;
    if (Z) {
        const Pack<T, VW> z = ld<T, VW>(Z + row * C + lane * VW);
#pragma unroll
        for (int e = 0; e < VW; ++e) out.e[e] = from_acc<T>(alpha * acc[e] + beta * to_acc(z.e[e]));
    } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) out.e[e] = from_acc<T>(alpha * acc[e]);
    }
    st<T, VW>(Y + row * C + lane * VW, out);
}

// Split-row SpMM for long rows (coarse levels): each row is shared by G lane
// groups (G * LPR threads); group g accumulates entries k0 + g, k0 + g + G, ...
// and the G partial rows are summed in LDS in a fixed order.
template <typename T, typename TV, int C, int G, bool SETS>
__global__ __launch_bounds__(kBlock) void k_spmm_split(int64_t n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const TV* __restrict__ va, const T* __restrict__ X,
                                                       T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta, int vs,
                                                       int m, OuterDiag sigma, int S, const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    using L = Lanes<T, C>;
    using TC = acc_t<T>;
    constexpr int VW = L::VW;
    constexpr int TPR = G * L::LPR;             // threads per row
    constexpr int RPB = kBlock / TPR;           // rows per block
    __shared__ TC sm[kBlock * VW];
    const int slot = threadIdx.x / TPR;
    const int g = (threadIdx.x % TPR) / L::LPR;
    const int lane = threadIdx.x % L::LPR;
    const int64_t row = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * RPB + slot;
    TC acc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = TC(0);
    if (row < n) {
        if constexpr (SETS) {
            int set[VW];
            if (column_sets<VW>(lane, vs, m, set))
                row_accumulate<T, C, VW, TV, true>(rp[row] + g, rp[row + 1], G, ci, va + set[0], X, lane, acc, vs);
            else
                row_accumulate_sets<T, C, VW, TV>(rp[row] + g, rp[row + 1], G, ci, va, X, lane, acc, vs, set);
        } else {
            row_accumulate<T, C, VW, TV>(rp[row] + g, rp[row + 1], G, ci, va, X, lane, acc);
        }
    }
#pragma unroll
    for (int e = 0; e < VW; ++e) sm[threadIdx.x * VW + e] = acc[e];
    __syncthreads();
    if (g == 0 && row < n) {
        // sm index of (slot, group q, lane, e) = ((slot * G + q) * LPR + lane) * VW + e
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] = TC(0);
        for (int q = 0; q < G; ++q) {
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] += sm[((slot * G + q) * L::LPR + lane) * VW + e];
        }
        if (sigma.idx) {   // outer diagonal, as in k_spmm
            const int32_t q = sigma.idx[row];
            if (q >= 0) {
                const Pack<T, VW> x = ld<T, VW>(X + row * C + lane * VW);
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    const int a = (lane * VW + e) / m;
                    if (a < S) acc[e] += (TC)sigma.val[(int64_t)q * S + a] * to_acc(x.e[e]);
                }
            }
        }
        Pack<T, VW> out;
        if (Z) {
            const Pack<T, VW> z = ld<T, VW>(Z + row * C + lane * VW);
#pragma unroll
            for (int e = 0; e < VW; ++e) out.e[e] = from_acc<T>(alpha * acc[e] + beta * to_acc(z.e[e]));
        } else {
#pragma unroll
            for (int e = 0; e < VW; ++e) out.e[e] = from_acc<T>(alpha * acc[e]);
        }
        st<T, VW>(Y + row * C + lane * VW, out);
    }
}

// ------------------------------------------------------------------ per-column dots
// partial[block * C + c] = sum over this block's rows of X[row, c] * Y[row, c]
// (FP64 accumulation); rows are visited grid-stride, the in-block reduction
// runs over row slots in a fixed order, so results are deterministic.
template <typename T, int C>
__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, const T* __restrict__ X,
                                                const T* __restrict__ Y, double* __restrict__ partial) {
    using L = Lanes<T, C>;
    constexpr int VW = L::VW;
    __shared__ double sm[kBlock * VW];
    const int slot = threadIdx.x / L::LPR;
    const int lane = threadIdx.x % L::LPR;
    double acc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * L::RPB + slot; row < n; row += (int64_t)gridDim.x * L::RPB) {
        const Pack<T, VW> x = ld<T, VW>(X + row * C + lane * VW);
        const Pack<T, VW> y = ld<T, VW>(Y + row * C + lane * VW);
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] += (double)x.e[e] * (double)y.e[e];
    }
#pragma unroll
    for (int e = 0; e < VW; ++e) sm[threadIdx.x * VW + e] = acc[e];
    __syncthreads();
    if (threadIdx.x < C) {
        double s = 0.0;
        for (int r = 0; r < L::RPB; ++r) s += sm[r * C + threadIdx.x];
        partial[(int64_t)blockIdx.x * C + threadIdx.x] = s;
    }
}

// out[o] = sum over nb blocks of partial[b * O + o]; one block per output o.
__global__ __launch_bounds__(kBlock) void k_reduce_partials(int nb, int O, const double* __restrict__ partial,
                                                            double* __restrict__ out) {
    __shared__ double sm[kBlock];
    const double s = block_sum_partials(nb, O, blockIdx.x, partial, sm);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// p = z + beta p on active columns
template <int C>
__global__ __launch_bounds__(kBlock) void k_pcg_pupdate(int64_t n, double* __restrict__ x, double* __restrict__ p,
                                                        const double* __restrict__ z,
                                                        const double* __restrict__ alpha,
                                                        const double* __restrict__ beta,
                                                        const int* __restrict__ active, int gated) {
    if (alpha_gate_closed(alpha, gated != 0)) return;
    using L = Lanes<double, C>;
    constexpr int VW = L::VW;
    const int64_t row = (int64_t)blockIdx.x * L::RPB + threadIdx.x / L::LPR;
    const int lane = threadIdx.x % L::LPR;
    if (row >= n) return;
    const int64_t o = row * C + lane * VW;
    Pack<double, VW> pv = ld<double, VW>(p + o);
    Pack<double, VW> xv = ld<double, VW>(x + o);
    const Pack<double, VW> zv = ld<double, VW>(z + o);
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        const int c = lane * VW + e;
        xv.e[e] += alpha[c] * pv.e[e];   // this iteration's x step (alpha = 0 on frozen columns)
        if (active[c]) pv.e[e] = zv.e[e] + beta[c] * pv.e[e];
    }
    st<double, VW>(x + o, xv);
    st<double, VW>(p + o, pv);
}

// ------------------------------------------------------------------ Q_s (Alg. 1, eq. (2.12))
// Q_s = 2^{-s/2} Had (x) I: a Walsh-Hadamard butterfly over the 2^s images of
// each base cell, fused with the layout change between the caller's n x m
// column-major vectors and the n_b x C multivector (column a*m + j).
template <int S>
__device__ __forceinline__ void fwht(double* v) {
#pragma unroll
    for (int h = 1; h < S; h <<= 1)
#pragma unroll
        for (int i = 0; i < S; ++i)
            if ((i & h) == 0) {
                const double u = v[i], w = v[i + h];
                v[i] = u + w;
                v[i + h] = u - w;
            }
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_qs_forward(int64_t n_b, int m, int C, int64_t n,
                                                       const int64_t* __restrict__ img,
                                                       const double* __restrict__ b, double* __restrict__ out,
                                                       double scale) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_b * m) return;
    const int64_t i = t / m;
    const int j = (int)(t % m);
    double v[S];
#pragma unroll
    for (int a = 0; a < S; ++a) v[a] = b[img[i * S + a] + (int64_t)j * n];
    fwht<S>(v);
#pragma unroll
    for (int a = 0; a < S; ++a) out[i * C + a * m + j] = scale * v[a];
}

// p != nullptr: the transform reads xh + alpha p (an x step not yet applied).
template <int S>
__global__ __launch_bounds__(kBlock) void k_qs_backward(int64_t n_b, int m, int C, int64_t n,
                                                        const int64_t* __restrict__ img,
                                                        const double* __restrict__ xh, double* __restrict__ x,
                                                        double scale, const double* __restrict__ p,
                                                        const double* __restrict__ alpha) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_b * m) return;
    const int64_t i = t / m;
    const int j = (int)(t % m);
    double v[S];
#pragma unroll
    for (int a = 0; a < S; ++a) {
        v[a] = xh[i * C + a * m + j];
        if (p) v[a] += alpha[a * m + j] * p[i * C + a * m + j];
    }
    fwht<S>(v);
#pragma unroll
    for (int a = 0; a < S; ++a) x[img[i * S + a] + (int64_t)j * n] = scale * v[a];
}

// per-RHS squared norms of the caller's b: block (x, j) sums a grid-stride
// share of column j and writes partial[x * m + j]; fixed-order tree in the block.
__global__ __launch_bounds__(kBlock) void k_colnorm2(int64_t n, int m, const double* __restrict__ b,
                                                     double* __restrict__ partial) {
    __shared__ double sm[kBlock];
    const int j = blockIdx.y;
    double s = 0.0;
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n; g += (int64_t)gridDim.x * kBlock) {
        const double v = b[g + (int64_t)j * n];
        s += v * v;
    }
    sm[threadIdx.x] = s;
    __syncthreads();
    for (unsigned w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * m + j] = sm[0];
}

// thresholds per column a*m + j: tol * ||b_j|| / sqrt(2^s); padded columns never start
__global__ void k_thresholds(int C, int S, int m, double tol, const double* __restrict__ bn2,
                             double* __restrict__ thr) {
    const int c = threadIdx.x;
    if (c < C) thr[c] = (c < S * m) ? tol * sqrt(bn2[c % m]) / sqrt((double)S) : INFINITY;
}

// ------------------------------------------------------------------ dense coarsest level
// X = Minv Y in FP64 (Y, X of type T), split over k: block (bx, ks) computes
// RB = 256 / LPR consecutive rows for k in chunk ks, staging the RB x KT slab
// of Minv and the KT x C slab of Y in LDS per tile; the FP64 partial rows go
// to part[ks] and a second kernel sums the chunks in a fixed order.
template <typename T, int C>
__global__ __launch_bounds__(kBlock) void k_dense_part(int64_t nL, int64_t kchunk, const double* __restrict__ Minv,
                                                       const T* __restrict__ y, double* __restrict__ part,
                                                       const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    using L = Lanes<T, C>;
    constexpr int VW = L::VW, LPR = L::LPR, RB = L::RPB;
    constexpr int KT = 32;
    __shared__ double sM[RB * KT];
    __shared__ T sY[KT * C];
    const int r = threadIdx.x / LPR, lane = threadIdx.x % LPR;
    const int64_t row0 = (int64_t)blockIdx.x * RB;
    const int64_t kb = (int64_t)blockIdx.y * kchunk;
    const int64_t ke = kb + kchunk < nL ? kb + kchunk : nL;
    double acc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = 0.0;
    for (int64_t k0 = kb; k0 < ke; k0 += KT) {
        for (int q = threadIdx.x; q < RB * KT; q += kBlock) {
            const int rr = q / KT, kk = q % KT;
            const int64_t gi = row0 + rr, gk = k0 + kk;
            sM[q] = (gi < nL && gk < ke) ? Minv[gi * nL + gk] : 0.0;
        }
        for (int q = threadIdx.x; q < KT * C; q += kBlock) {
            const int64_t gk = k0 + q / C;
            sY[q] = gk < ke ? y[gk * C + q % C] : T{};
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < KT; ++kk) {
            const double a = sM[r * KT + kk];
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] += a * (double)to_acc(sY[kk * C + lane * VW + e]);
        }
        __syncthreads();
    }
    if (row0 + r < nL) {
        double* o = part + ((int64_t)blockIdx.y * nL + row0 + r) * C + lane * VW;
#pragma unroll
        for (int e = 0; e < VW; ++e) o[e] = acc[e];
    }
}

// yp[(a * ldm + k) * MP + j] = y[k, a*m + j] (zero for j >= m or k >= nL):
// every subsystem's m columns packed contiguously, ldm rows per subsystem,
// for the dense solves below.
template <typename T, int MP>
__global__ __launch_bounds__(kBlock) void k_pack_sets(int64_t nL, int64_t ldm, int C, int S, int m,
                                                      const T* __restrict__ y, T* __restrict__ yp,
                                                      const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)S * ldm * MP) return;
    const int j = (int)(idx % MP);
    const int64_t ak = idx / MP;
    const int a = (int)(ak / ldm);
    const int64_t k = ak % ldm;
    yp[idx] = j < m && k < nL ? y[k * C + a * m + j] : T{};
}

// Per-subsystem coarsest solves: out[:, a*m + j] = Minv_a y[:, a*m + j] for
// subsystem a = blockIdx.y with its own inverse Minv + a * nL * ldm (rows of
// ldm entries, the ones past nL zero).  With only m columns per inverse this
// is a bandwidth-bound batched GEMV: each wavefront owns R rows, its lanes
// walk k in steps of 64 * KV (KV consecutive entries per lane, so every row
// is read as coalesced 512- or 1024-byte segments and every entry of the
// inverses once; the right-hand sides come packed, MP values per k
// contiguous), the sums are kept in FP64, and the per-lane partial sums are
// reduced across the wave by a fixed butterfly.  Blocks of the last subsystem
// also clear the padded columns >= S * m.
template <typename T, typename TM, int MP, int R>
__global__ __launch_bounds__(kBlock) void k_dense_sets(int64_t nL, int64_t ldm, int C, int S, int m,
                                                       const TM* __restrict__ Minv, const T* __restrict__ yp,
                                                       T* __restrict__ out, const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    constexpr int W = 64;
    constexpr int KV = sizeof(TM) == 4 ? 4 : 1;                                   // inverse entries per lane load
    constexpr int PW = (MP * (int)sizeof(T)) >= 16 ? 16 / (int)sizeof(T) : MP;   // values per packed load
    const int wave = threadIdx.x / W, lane = threadIdx.x % W;
    const int a = blockIdx.y;
    const int64_t row0 = ((int64_t)blockIdx.x * (kBlock / W) + wave) * R;
    if (row0 >= nL) return;   // the whole wavefront leaves together
    const TM* Ma = Minv + (int64_t)a * nL * ldm;
    const T* ya = yp + (int64_t)a * ldm * MP;
    double acc[R][MP];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < MP; ++j) acc[r][j] = 0.0;
#pragma unroll 4
    for (int64_t k0 = (int64_t)lane * KV; k0 < ldm; k0 += W * KV) {
        Pack<TM, KV> mv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (row0 + r < nL) {
                mv[r] = ld_stream<TM, KV>(Ma + (row0 + r) * ldm + k0);
            } else {
#pragma unroll
                for (int e = 0; e < KV; ++e) mv[r].e[e] = TM(0);
            }
        }
#pragma unroll
        for (int kk = 0; kk < KV; ++kk) {
            double xv[MP];
#pragma unroll
            for (int q = 0; q < MP; q += PW) {
                const Pack<T, PW> v = ld<T, PW>(ya + (k0 + kk) * MP + q);
#pragma unroll
                for (int e = 0; e < PW; ++e) xv[q + e] = (double)to_acc(v.e[e]);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double mvd = (double)mv[r].e[kk];
#pragma unroll
                for (int j = 0; j < MP; ++j) acc[r][j] += mvd * xv[j];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < MP; ++j) {
            double v = acc[r][j];
#pragma unroll
            for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
            acc[r][j] = v;
        }
    // lane r * MP + j writes row r, column j (R * MP <= 64)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < MP; ++j)
            if (lane == r * MP + j && j < m && row0 + r < nL) out[(row0 + r) * C + a * m + j] = from_double<T>(acc[r][j]);
    if (a == S - 1) {
        const int pad = C - S * m;
        for (int q = lane; q < R * pad; q += W) {
            const int64_t i = row0 + q / pad;
            if (i < nL) out[i * C + S * m + q % pad] = T{};
        }
    }
}

// out[i] = sum over the ks chunks; columns >= ncol (never written by the
// per-subsystem solve) are set to zero.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_sum(int64_t len, int ks, int C, int ncol,
                                                      const double* __restrict__ part, T* __restrict__ out,
                                                      const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    if ((int)(i % C) < ncol)
        for (int q = 0; q < ks; ++q) s += part[(int64_t)q * len + i];
    out[i] = from_double<T>(s);
}

// ------------------------------------------------------------------ elementwise
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t len, T* __restrict__ p, T v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) p[i] = v;
}

template <typename TO, typename TI>
__global__ __launch_bounds__(kBlock) void k_cast(int64_t len, const TI* __restrict__ a, TO* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) b[i] = from_double<TO>(static_cast<double>(to_acc(a[i])));
}

// ------------------------------------------------------------------ column-wise vector ops
// X[:, c] *= f[c]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_cols(int64_t len, int C, T* __restrict__ X,
                                                       const double* __restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) X[i] = (T)((double)X[i] * f[i % C]);
}

// Y[:, c] -= h[c] * X[:, c]
__global__ __launch_bounds__(kBlock) void k_axpy_cols(int64_t len, int C, double* __restrict__ Y,
                                                      const double* __restrict__ X, const double* __restrict__ h) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) Y[i] -= h[i % C] * X[i];
}

// ------------------------------------------------------------------ low-rank corrections
// U is n x (S * k) row-major: U[i, a*k + t] is entry i of correction vector t
// of subsystem a.  Subsystem a owns multivector columns a*m .. a*m + m - 1.

// U[i, a*k + t] = sum_j V_j[i, a] * cm[(a*K + j)*k + t] (Ritz vectors from the
// Lanczos basis V_j, stored n x C with C >= S, one column per subsystem).
template <typename TU>
__global__ __launch_bounds__(kBlock) void k_lrc_combine(int64_t n, int S, int k, int K, int C,
                                                        const double* __restrict__ V,
                                                        const double* __restrict__ cm, TU* __restrict__ U) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= n * S * k) return;
    const int64_t i = idx / (S * k);
    const int at = (int)(idx % (S * k));
    const int a = at / k, t = at % k;
    double s = 0.0;
    for (int j = 0; j < K; ++j) s += V[((int64_t)j * n + i) * C + a] * cm[((int64_t)a * K + j) * k + t];
    U[idx] = from_double<TU>(s);
}

// partial[b, o] = sum over block b's rows of U[i, a*k+t] * R[i, a*m+j],
// o = (a*k + t)*m + j.  Rows are split into gridDim.x contiguous chunks.
template <typename TU>
__global__ __launch_bounds__(kBlock) void k_lrc_project(int64_t n, int S, int k, int m, int C,
                                                        const TU* __restrict__ U, const double* __restrict__ R,
                                                        double* __restrict__ partial) {
    const int O = S * k * m;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
    for (int o = threadIdx.x; o < O; o += kBlock) {
        const int j = o % m;
        const int at = o / m;
        const int a = at / k;
        double s = 0.0;
        for (int64_t i = r0; i < r1; ++i)
            s += (double)to_acc(U[i * (S * k) + at]) * R[i * C + a * m + j];
        partial[(int64_t)blockIdx.x * O + o] = s;
    }
}

// W[o] = coef[o / m] * sum_b partial[b, o]  (fixed order over b; o = (a*k + t)*m + j)
__global__ __launch_bounds__(kBlock) void k_lrc_finish(int nb, int O, int m,
                                                       const double* __restrict__ partial,
                                                       const double* __restrict__ coef, double* __restrict__ W) {
    const int o = blockIdx.x * kBlock + threadIdx.x;
    if (o >= O) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * O + o];
    W[o] = coef[o / m] * s;
}

// Z[i, a*m+j] += sum_t U[i, a*k+t] * W[(a*k+t)*m + j] for columns < S*m
template <typename TU>
__global__ __launch_bounds__(kBlock) void k_lrc_expand(int64_t n, int S, int k, int m, int C,
                                                       const TU* __restrict__ U, const double* __restrict__ W,
                                                       double* __restrict__ Z) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= n * C) return;
    const int64_t i = idx / C;
    const int col = (int)(idx % C);
    if (col >= S * m) return;
    const int a = col / m, j = col % m;
    double s = 0.0;
    const TU* u = U + i * (S * k) + a * k;
    for (int t = 0; t < k; ++t) s += (double)to_acc(u[t]) * W[(a * k + t) * m + j];
    Z[idx] += s;
}

// ------------------------------------------------------------------ adjoint gradient
// grad[i] = sum over the faces of base cell i, the images a and the right-hand
// sides j of g_f dT_f/dkappa_i, with g_f = -(lam_u - lam_v)(p_u - p_v) for
// interior and mirror faces and -lam_u p_u for wall faces (lam, p: n x m
// column-major in the caller's ordering).  One thread per base cell, faces in
// a fixed order: deterministic, no atomics.
__global__ __launch_bounds__(kBlock) void k_kappa_grad(int64_t n_b, int S, int64_t n, int m,
                                                       const int64_t* __restrict__ cfp,
                                                       const int32_t* __restrict__ cfi,
                                                       const int64_t* __restrict__ img,
                                                       const int64_t* __restrict__ ca, const int64_t* __restrict__ cb,
                                                       const int8_t* __restrict__ kind,
                                                       const int8_t* __restrict__ axis,
                                                       const double* __restrict__ area,
                                                       const double* __restrict__ da, const double* __restrict__ db,
                                                       const double* __restrict__ kap,
                                                       const double* __restrict__ lam, const double* __restrict__ p,
                                                       double* __restrict__ grad) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_b) return;
    const double ki = kap[i];
    double acc = 0.0;
    for (int64_t e = cfp[i]; e < cfp[i + 1]; ++e) {
        const int64_t q = cfi[e];
        const int K = kind[q];
        if (K == 0) {
            const bool first = ca[q] == i;
            const int64_t o = first ? cb[q] : ca[q];
            const double di = first ? da[q] : db[q], dout = first ? db[q] : da[q];
            const double T = area[q] / (di / ki + dout / kap[o]);
            const double dT = T * T * di / (area[q] * ki * ki);
            for (int a = 0; a < S; ++a)
                for (int j = 0; j < m; ++j) {
                    const int64_t u = img[i * S + a] + (int64_t)j * n, v = img[o * S + a] + (int64_t)j * n;
                    acc += -(lam[u] - lam[v]) * (p[u] - p[v]) * dT;
                }
        } else if (K == 1) {
            const double dT = area[q] / da[q];
            for (int a = 0; a < S; ++a)
                for (int j = 0; j < m; ++j) {
                    const int64_t u = img[i * S + a] + (int64_t)j * n;
                    acc += -lam[u] * p[u] * dT;
                }
        } else {
            const int bit = 1 << axis[q];
            const double dT = area[q] / (2.0 * da[q]);
            for (int a = 0; a < S; ++a) {
                if (a & bit) continue;   // each mirror pair once
                for (int j = 0; j < m; ++j) {
                    const int64_t u = img[i * S + a] + (int64_t)j * n, v = img[i * S + (a ^ bit)] + (int64_t)j * n;
                    acc += -(lam[u] - lam[v]) * (p[u] - p[v]) * dT;
                }
            }
        }
    }
    grad[i] = acc;
}

// pub[0..1] = flags[0..1], then pub[2] = seq: a solve's flags published to
// fine-grained host memory; the sequence number is stored last, after a
// system-scope fence, so a host that sees seq also sees the flags.
__global__ void k_publish_flags(const int* __restrict__ flags, int* pub, int seq) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        volatile int* v = pub;
        v[0] = flags[0];
        v[1] = flags[1];
        __threadfence_system();
        v[2] = seq;
        __threadfence_system();
    }
}

// out[2i], out[2i+1] = breakdown flag and active-column count of system i
__global__ void k_gather_flags(int nsys, int* const* __restrict__ ptrs, int* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nsys) {
        out[2 * i] = ptrs[i][0];
        out[2 * i + 1] = ptrs[i][1];
    }
}

// ------------------------------------------------------------------ allocation-free workspace
// The workspace of msp_solve_device_noalloc lives in this file-scope device
// array: every GPU the library runs on holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol); it takes the device address from
// hipGetSymbolAddress, looked up once per device with that device current.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

hipError_t scratch_init() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
    return hipSuccess;
}

void* scratch_address(int device) {
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

// ------------------------------------------------------------------ host launchers


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

// value sets are supported for FP64 and FP32 values (not bfloat16)
template <typename TV>
constexpr bool sets_ok() {
    return !std::is_same<TV, Bf16>::value;
}

template <typename T, typename TV>
hipError_t launch_spmm(hipStream_t st, int C, int64_t n, const int32_t* rp, const int32_t* ci, const TV* va,
                       const T* X, T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta, OuterDiag sigma, int S, int m,
                       int vs, bool wide, const int* gate) {
    if (n <= 0) return hipSuccess;
    if (vs > 1 && (!sets_ok<TV>() || m < 1)) return hipErrorInvalidValue;
    MSP_DISPATCH_C(C, {
        using L = Lanes<T, CC>;
        if constexpr (sets_ok<TV>()) {
            if (vs > 1) {
                hipLaunchKernelGGL((k_spmm<T, TV, CC, true, false>), dim3(blocks_for(n, L::RPB)), dim3(kBlock), 0, st,
                                   n, rp, ci, va, X, Y, Z, alpha, beta, sigma, S, m, vs, gate);
                break;
            }
        }
        using LW = Lanes<T, CC, true>;
        if (wide && LW::VW != L::VW) {
            hipLaunchKernelGGL((k_spmm<T, TV, CC, false, true>), dim3(blocks_for(n, LW::RPB)), dim3(kBlock), 0, st, n,
                               rp, ci, va, X, Y, Z, alpha, beta, sigma, S, m, 1, gate);
            break;
        }
        hipLaunchKernelGGL((k_spmm<T, TV, CC, false, false>), dim3(blocks_for(n, L::RPB)), dim3(kBlock), 0, st, n, rp,
                           ci, va, X, Y, Z, alpha, beta, sigma, S, m, 1, gate);
    });
    return hipGetLastError();
}

bool spmm_has_wide(int C, int elem_bytes) {
    const int vw = lane_width(elem_bytes), ww = 16 / elem_bytes;
    return (ww < C ? ww : C) != (vw < C ? vw : C);
}

template <typename T, typename TV, int CC, int G>
static void launch_split(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci, const TV* va, const T* X,
                         T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta, int vs, int m, OuterDiag sigma, int S,
                         const int* gate) {
    constexpr int TPR = G * Lanes<T, CC>::LPR;
    if constexpr (TPR <= kBlock) {
        constexpr int RPB = kBlock / TPR;
        if constexpr (sets_ok<TV>()) {
            if (vs > 1) {
                hipLaunchKernelGGL((k_spmm_split<T, TV, CC, G, true>), dim3(blocks_for(n, RPB)), dim3(kBlock), 0, st,
                                   n, rp, ci, va, X, Y, Z, alpha, beta, vs, m, sigma, S, gate);
                return;
            }
        }
        hipLaunchKernelGGL((k_spmm_split<T, TV, CC, G, false>), dim3(blocks_for(n, RPB)), dim3(kBlock), 0, st, n, rp,
                           ci, va, X, Y, Z, alpha, beta, 1, m, sigma, S, gate);
    }
}

template <typename T, typename TV>
hipError_t launch_spmm_split(hipStream_t st, int C, int G, int64_t n, const int32_t* rp, const int32_t* ci,
                             const TV* va, const T* X, T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta, int vs, int m,
                             OuterDiag sigma, int S, const int* gate) {
    if (n <= 0) return hipSuccess;
    if ((vs > 1 || sigma.idx) && m < 1) return hipErrorInvalidValue;
    if (vs > 1 && !sets_ok<TV>()) return hipErrorInvalidValue;
    MSP_DISPATCH_C(C, {
        constexpr int LPR = Lanes<T, CC>::LPR;
        const int gmax = kBlock / LPR;
        const int g = G < gmax ? G : gmax;
        switch (g) {
            case 2: launch_split<T, TV, CC, 2>(st, n, rp, ci, va, X, Y, Z, alpha, beta, vs, m, sigma, S, gate); break;
            case 4: launch_split<T, TV, CC, 4>(st, n, rp, ci, va, X, Y, Z, alpha, beta, vs, m, sigma, S, gate); break;
            case 8: launch_split<T, TV, CC, 8>(st, n, rp, ci, va, X, Y, Z, alpha, beta, vs, m, sigma, S, gate); break;
            case 16: launch_split<T, TV, CC, 16>(st, n, rp, ci, va, X, Y, Z, alpha, beta, vs, m, sigma, S, gate); break;
            case 32: launch_split<T, TV, CC, 32>(st, n, rp, ci, va, X, Y, Z, alpha, beta, vs, m, sigma, S, gate); break;
            case 64: launch_split<T, TV, CC, 64>(st, n, rp, ci, va, X, Y, Z, alpha, beta, vs, m, sigma, S, gate); break;
            default: launch_split<T, TV, CC, 1>(st, n, rp, ci, va, X, Y, Z, alpha, beta, vs, m, sigma, S, gate); break;
        }
    });
    return hipGetLastError();
}

#define MSP_SPMM_INST(T, TV)                                                                                         \
    template hipError_t launch_spmm<T, TV>(hipStream_t, int, int64_t, const int32_t*, const int32_t*, const TV*,     \
                                           const T*, T*, const T*, acc_t<T>, acc_t<T>, OuterDiag, int, int, int,      \
                                           bool, const int*);                                                          \
    template hipError_t launch_spmm_split<T, TV>(hipStream_t, int, int, int64_t, const int32_t*, const int32_t*,     \
                                                 const TV*, const T*, T*, const T*, acc_t<T>, acc_t<T>, int, int,   \
                                                 OuterDiag, int, const int*);
MSP_SPMM_INST(double, double)
MSP_SPMM_INST(float, float)
MSP_SPMM_INST(float, Bf16)
MSP_SPMM_INST(Bf16, float)

template <typename T>
hipError_t launch_dot(hipStream_t st, int C, int64_t n, const T* X, const T* Y, double* partial, int nb,
                      double* out) {
    MSP_DISPATCH_C(C, {
        hipLaunchKernelGGL((k_dot<T, CC>), dim3(nb), dim3(kBlock), 0, st, n, X, Y, partial);
        hipLaunchKernelGGL(k_reduce_partials, dim3(CC), dim3(kBlock), 0, st, nb, CC, partial, out);
    });
    return hipGetLastError();
}
template hipError_t launch_dot<double>(hipStream_t, int, int64_t, const double*, const double*, double*, int,
                                       double*);
template hipError_t launch_dot<float>(hipStream_t, int, int64_t, const float*, const float*, double*, int,
                                      double*);

hipError_t launch_pcg_pupdate(hipStream_t st, int C, int64_t n, double* x, double* p, const double* z,
                              const double* alpha, const double* beta, const int* active, bool gated) {
    MSP_DISPATCH_C(C, {
        using L = Lanes<double, CC>;
        hipLaunchKernelGGL((k_pcg_pupdate<CC>), dim3(blocks_for(n, L::RPB)), dim3(kBlock), 0, st, n, x, p, z, alpha,
                           beta, active, gated ? 1 : 0);
    });
    return hipGetLastError();
}
#define MSP_DISPATCH_S(S, ...)                                   \
    switch (S) {                                                 \
        case 1: { constexpr int SS = 1; __VA_ARGS__; } break;    \
        case 2: { constexpr int SS = 2; __VA_ARGS__; } break;    \
        case 4: { constexpr int SS = 4; __VA_ARGS__; } break;    \
        case 8: { constexpr int SS = 8; __VA_ARGS__; } break;    \
        case 16: { constexpr int SS = 16; __VA_ARGS__; } break;  \
        case 32: { constexpr int SS = 32; __VA_ARGS__; } break;  \
        case 64: { constexpr int SS = 64; __VA_ARGS__; } break;  \
        default: return hipErrorInvalidValue;                    \
    }

hipError_t launch_qs_forward(hipStream_t st, int S, int64_t n_b, int m, int C, int64_t n, const int64_t* img,
                             const double* b, double* out) {
    const double scale = 1.0 / std::sqrt((double)S);
    MSP_DISPATCH_S(S, {
        hipLaunchKernelGGL((k_qs_forward<SS>), dim3(blocks_for(n_b * m, kBlock)), dim3(kBlock), 0, st, n_b, m, C,
                           n, img, b, out, scale);
    });
    return hipGetLastError();
}
hipError_t launch_qs_backward(hipStream_t st, int S, int64_t n_b, int m, int C, int64_t n, const int64_t* img,
                              const double* xh, double* x, const double* p, const double* alpha) {
    if (p && !alpha) return hipErrorInvalidValue;
    const double scale = 1.0 / std::sqrt((double)S);
    MSP_DISPATCH_S(S, {
        hipLaunchKernelGGL((k_qs_backward<SS>), dim3(blocks_for(n_b * m, kBlock)), dim3(kBlock), 0, st, n_b, m, C,
                           n, img, xh, x, scale, p, alpha);
    });
    return hipGetLastError();
}
hipError_t launch_colnorm2(hipStream_t st, int64_t n, int m, const double* b, double* partial, int nb,
                           double* out) {
    hipLaunchKernelGGL(k_colnorm2, dim3(nb, m), dim3(kBlock), 0, st, n, m, b, partial);
    hipLaunchKernelGGL(k_reduce_partials, dim3(m), dim3(kBlock), 0, st, nb, m, partial, out);
    return hipGetLastError();
}
hipError_t launch_thresholds(hipStream_t st, int C, int S, int m, double tol, const double* bn2, double* thr) {
    hipLaunchKernelGGL(k_thresholds, dim3(1), dim3(64), 0, st, C, S, m, tol, bn2, thr);
    return hipGetLastError();
}

// k-chunks of the dense product: about 1024 blocks in total, whole tiles per chunk
int dense_splits(int C, int64_t nL, int elem_bytes) {
    const int vw = lane_width(elem_bytes);
    const int lpr = C >= vw ? C / vw : 1;   // lanes per row of Lanes<T, C> for a T of elem_bytes
    const int64_t rb = kBlock / lpr;
    const int64_t rows = (nL + rb - 1) / rb;
    int64_t ks = (1024 + rows - 1) / rows;
    const int64_t tiles = (nL + 31) / 32;
    if (ks > tiles) ks = tiles;
    if (ks < 1) ks = 1;
    if (ks > 64) ks = 64;
    return (int)ks;
}

template <typename T>
hipError_t launch_dense(hipStream_t st, int C, int64_t nL, const double* Minv, const T* y, T* out, double* part,
                        const int* gate) {
    const int ks = dense_splits(C, nL, (int)sizeof(T));
    const int64_t tiles = (nL + 31) / 32;
    const int64_t kchunk = ((tiles + ks - 1) / ks) * 32;
    MSP_DISPATCH_C(C, {
        using L = Lanes<T, CC>;
        hipLaunchKernelGGL((k_dense_part<T, CC>), dim3(blocks_for(nL, L::RPB), ks), dim3(kBlock), 0, st, nL, kchunk,
                           Minv, y, part, gate);
        hipLaunchKernelGGL((k_dense_sum<T>), dim3(blocks_for(nL * CC, kBlock)), dim3(kBlock), 0, st, nL * CC, ks, CC,
                           CC, part, out, gate);
    });
    return hipGetLastError();
}
template hipError_t launch_dense<double>(hipStream_t, int, int64_t, const double*, const double*, double*, double*,
                                             const int*);
template hipError_t launch_dense<float>(hipStream_t, int, int64_t, const double*, const float*, float*, double*,
                                             const int*);
template hipError_t launch_dense<Bf16>(hipStream_t, int, int64_t, const double*, const Bf16*, Bf16*, double*,
                                             const int*);

static int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

template <typename T, typename TM, int MP, int R>
static void launch_dense_sets_r(hipStream_t st, int C, int S, int m, int64_t nL, int64_t ldm, const TM* Minv,
                                const T* yp, T* out, const int* gate) {
    if constexpr (R * MP <= 64) {
        const int64_t rows_per_block = (int64_t)(kBlock / 64) * R;
        hipLaunchKernelGGL((k_dense_sets<T, TM, MP, R>), dim3(blocks_for(nL, (int)rows_per_block), S), dim3(kBlock),
                           0, st, nL, ldm, C, S, m, Minv, yp, out, gate);
    }
}

template <typename T, typename TM, int MP>
static void launch_dense_sets_mp(hipStream_t st, int C, int S, int m, int64_t nL, int64_t ldm, const TM* Minv,
                                 const T* y, T* out, T* yp, int R, const int* gate) {
    hipLaunchKernelGGL((k_pack_sets<T, MP>), dim3(blocks_for((int64_t)S * ldm * MP, kBlock)), dim3(kBlock), 0, st, nL,
                       ldm, C, S, m, y, yp, gate);
    switch (R) {
        case 8: launch_dense_sets_r<T, TM, MP, 8>(st, C, S, m, nL, ldm, Minv, yp, out, gate); break;
        case 4: launch_dense_sets_r<T, TM, MP, 4>(st, C, S, m, nL, ldm, Minv, yp, out, gate); break;
        case 2: launch_dense_sets_r<T, TM, MP, 2>(st, C, S, m, nL, ldm, Minv, yp, out, gate); break;
        default: launch_dense_sets_r<T, TM, MP, 1>(st, C, S, m, nL, ldm, Minv, yp, out, gate); break;
    }
}

int dense_sets_rows_max(int m) {
    const int mp = pow2_at_least(m);
    return mp <= 8 ? 8 : 64 / mp;
}

int64_t dense_sets_ld(int64_t nL, int minv_bytes) { return minv_bytes == 4 ? (nL + 3) / 4 * 4 : nL; }

template <typename T, typename TM>
hipError_t launch_dense_sets(hipStream_t st, int C, int S, int m, int64_t nL, const TM* Minv, const T* y,
                             T* out, T* yp, int R, const int* gate) {
    if (S * m > C || m < 1 || m > 64 || S < 1) return hipErrorInvalidValue;
    if (R != 1 && R != 2 && R != 4 && R != 8) return hipErrorInvalidValue;
    if (R > dense_sets_rows_max(m)) R = dense_sets_rows_max(m);
    if (nL <= 0) return hipSuccess;
    const int64_t ldm = dense_sets_ld(nL, (int)sizeof(TM));
    switch (pow2_at_least(m)) {
        case 1: launch_dense_sets_mp<T, TM, 1>(st, C, S, m, nL, ldm, Minv, y, out, yp, R, gate); break;
        case 2: launch_dense_sets_mp<T, TM, 2>(st, C, S, m, nL, ldm, Minv, y, out, yp, R, gate); break;
        case 4: launch_dense_sets_mp<T, TM, 4>(st, C, S, m, nL, ldm, Minv, y, out, yp, R, gate); break;
        case 8: launch_dense_sets_mp<T, TM, 8>(st, C, S, m, nL, ldm, Minv, y, out, yp, R, gate); break;
        case 16: launch_dense_sets_mp<T, TM, 16>(st, C, S, m, nL, ldm, Minv, y, out, yp, R, gate); break;
        case 32: launch_dense_sets_mp<T, TM, 32>(st, C, S, m, nL, ldm, Minv, y, out, yp, R, gate); break;
        default: launch_dense_sets_mp<T, TM, 64>(st, C, S, m, nL, ldm, Minv, y, out, yp, R, gate); break;
    }
    return hipGetLastError();
}
template hipError_t launch_dense_sets<double, double>(hipStream_t, int, int, int, int64_t, const double*,
                                                      const double*, double*, double*, int, const int*);
template hipError_t launch_dense_sets<float, float>(hipStream_t, int, int, int, int64_t, const float*, const float*,
                                                    float*, float*, int, const int*);
template hipError_t launch_dense_sets<Bf16, float>(hipStream_t, int, int, int, int64_t, const float*, const Bf16*,
                                                   Bf16*, Bf16*, int, const int*);
template hipError_t launch_dense_sets<float, double>(hipStream_t, int, int, int, int64_t, const double*,
                                                     const float*, float*, float*, int, const int*);
template hipError_t launch_dense_sets<Bf16, double>(hipStream_t, int, int, int, int64_t, const double*, const Bf16*,
                                                    Bf16*, Bf16*, int, const int*);

template <typename T>
hipError_t launch_fill(hipStream_t st, int64_t len, T* p, T v) {
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill<T>), dim3(blocks_for(len, kBlock)), dim3(kBlock), 0, st, len, p, v);
    return hipGetLastError();
}
template hipError_t launch_fill<double>(hipStream_t, int64_t, double*, double);
template hipError_t launch_fill<float>(hipStream_t, int64_t, float*, float);
template hipError_t launch_fill<int>(hipStream_t, int64_t, int*, int);
template hipError_t launch_fill<Bf16>(hipStream_t, int64_t, Bf16*, Bf16);

hipError_t launch_publish_flags(hipStream_t st, const int* flags, int* pub, int seq) {
    hipLaunchKernelGGL(k_publish_flags, dim3(1), dim3(64), 0, st, flags, pub, seq);
    return hipGetLastError();
}

hipError_t launch_gather_flags(hipStream_t st, int nsys, int* const* ptrs, int* out) {
    hipLaunchKernelGGL(k_gather_flags, dim3(blocks_for(nsys, 64)), dim3(64), 0, st, nsys, ptrs, out);
    return hipGetLastError();
}

hipError_t launch_kappa_grad(hipStream_t st, int64_t n_b, int S, int64_t n, int m, const int64_t* cfp,
                            const int32_t* cfi, const int64_t* img, const int64_t* ca, const int64_t* cb,
                            const int8_t* kind, const int8_t* axis, const double* area, const double* da,
                            const double* db, const double* kap, const double* lam, const double* p, double* grad) {
    hipLaunchKernelGGL(k_kappa_grad, dim3(blocks_for(n_b, kBlock)), dim3(kBlock), 0, st, n_b, S, n, m, cfp, cfi, img,
                       ca, cb, kind, axis, area, da, db, kap, lam, p, grad);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_cols(hipStream_t st, int64_t len, int C, T* X, const double* f) {
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_scale_cols<T>), dim3(blocks_for(len, kBlock)), dim3(kBlock), 0, st, len, C, X, f);
    return hipGetLastError();
}
template hipError_t launch_scale_cols<double>(hipStream_t, int64_t, int, double*, const double*);

hipError_t launch_axpy_cols(hipStream_t st, int64_t len, int C, double* Y, const double* X, const double* h) {
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy_cols, dim3(blocks_for(len, kBlock)), dim3(kBlock), 0, st, len, C, Y, X, h);
    return hipGetLastError();
}

template <typename TU>
hipError_t launch_lrc_combine(hipStream_t st, int64_t n, int S, int k, int K, int C, const double* V,
                              const double* cm, TU* U) {
    hipLaunchKernelGGL((k_lrc_combine<TU>), dim3(blocks_for(n * S * k, kBlock)), dim3(kBlock), 0, st, n, S, k, K,
                       C, V, cm, U);
    return hipGetLastError();
}
template hipError_t launch_lrc_combine<double>(hipStream_t, int64_t, int, int, int, int, const double*,
                                               const double*, double*);
template hipError_t launch_lrc_combine<float>(hipStream_t, int64_t, int, int, int, int, const double*,
                                              const double*, float*);
template hipError_t launch_lrc_combine<Bf16>(hipStream_t, int64_t, int, int, int, int, const double*,
                                             const double*, Bf16*);

template <typename TU>
hipError_t launch_lrc_apply(hipStream_t st, int64_t n, int S, int k, int m, int C, const TU* U, const double* R,
                            double* Z, const double* coef, double* partial, int nb, double* W) {
    const int O = S * k * m;
    hipLaunchKernelGGL((k_lrc_project<TU>), dim3(nb), dim3(kBlock), 0, st, n, S, k, m, C, U, R, partial);
    hipLaunchKernelGGL(k_lrc_finish, dim3(blocks_for(O, kBlock)), dim3(kBlock), 0, st, nb, O, m, partial, coef, W);
    hipLaunchKernelGGL((k_lrc_expand<TU>), dim3(blocks_for(n * C, kBlock)), dim3(kBlock), 0, st, n, S, k, m, C, U,
                       W, Z);
    return hipGetLastError();
}
template hipError_t launch_lrc_apply<double>(hipStream_t, int64_t, int, int, int, int, const double*, const double*,
                                             double*, const double*, double*, int, double*);
template hipError_t launch_lrc_apply<float>(hipStream_t, int64_t, int, int, int, int, const float*, const double*,
                                            double*, const double*, double*, int, double*);

template <typename TO, typename TI>
hipError_t launch_cast(hipStream_t st, int64_t len, const TI* a, TO* b) {
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_cast<TO, TI>), dim3(blocks_for(len, kBlock)), dim3(kBlock), 0, st, len, a, b);
    return hipGetLastError();
}
template hipError_t launch_cast<float, double>(hipStream_t, int64_t, const double*, float*);
template hipError_t launch_cast<double, float>(hipStream_t, int64_t, const float*, double*);
template hipError_t launch_cast<Bf16, double>(hipStream_t, int64_t, const double*, Bf16*);
template hipError_t launch_cast<double, Bf16>(hipStream_t, int64_t, const Bf16*, double*);

}  // namespace msp
