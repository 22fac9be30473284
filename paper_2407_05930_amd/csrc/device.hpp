// Device-side helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace msp {

// matrix value -> arithmetic type
template <typename T>
__device__ __forceinline__ T cvt(T v) {
    return v;
}
template <typename T>
__device__ __forceinline__ T cvt(Bf16 v);
template <>
__device__ __forceinline__ float cvt<float>(Bf16 v) {
    return __uint_as_float(static_cast<uint32_t>(v.bits) << 16);
}

// storage <-> arithmetic conversions (identity except for bfloat16)
__device__ __forceinline__ float to_acc(Bf16 v) { return cvt<float>(v); }
__device__ __forceinline__ float to_acc(float v) { return v; }
__device__ __forceinline__ double to_acc(double v) { return v; }
template <typename T>
__device__ __forceinline__ T from_acc(acc_t<T> v) {
    return v;
}
template <>
__device__ __forceinline__ Bf16 from_acc<Bf16>(float f) {   // round to nearest even (finite inputs)
    const uint32_t u = __float_as_uint(f);
    return Bf16{static_cast<uint16_t>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16)};
}
// a storage value from a double (casts at the boundary of the V-cycle)
template <typename T>
__device__ __forceinline__ T from_double(double v) {
    return from_acc<T>(static_cast<acc_t<T>>(v));
}

constexpr int kBlock = 256;

template <typename T, int VW>
struct alignas(sizeof(T) * VW) Pack {
    T e[VW];
};

template <typename T, int VW>
__device__ __forceinline__ Pack<T, VW> ld(const T* p) {
    return *reinterpret_cast<const Pack<T, VW>*>(p);
}
template <typename T, int VW>
__device__ __forceinline__ void st(T* p, const Pack<T, VW>& v) {
    *reinterpret_cast<Pack<T, VW>*>(p) = v;
}

// Streaming accesses (nontemporal hint) for data whose next use is further
// away than the memory-side cache reaches (the per-subsystem coarsest
// inverses, read once per V-cycle): they then do not displace the V-cycle's
// matrices and vectors, which are reused within a cycle.
template <int B>
struct NtWord;   // an integer vector of B bytes
template <>
struct NtWord<32> { typedef uint32_t type __attribute__((ext_vector_type(8))); };
template <>
struct NtWord<16> { typedef uint32_t type __attribute__((ext_vector_type(4))); };
template <>
struct NtWord<8> { typedef uint32_t type __attribute__((ext_vector_type(2))); };
template <>
struct NtWord<4> { typedef uint32_t type; };
template <>
struct NtWord<2> { typedef uint16_t type; };

template <typename T, int VW>
__device__ __forceinline__ Pack<T, VW> ld_stream(const T* p) {
    using W = typename NtWord<sizeof(Pack<T, VW>)>::type;
    const W w = __builtin_nontemporal_load(reinterpret_cast<const W*>(p));
    Pack<T, VW> v;
    __builtin_memcpy(&v, &w, sizeof(v));
    return v;
}

// Lane layout of an n x C row-major multivector: each row is handled by
// LPR = C / VW lanes with VW consecutive columns per lane (lane_width
// columns: 16-byte accesses, 8-byte for bfloat16, where the row is wide
// enough); a 256-thread block covers RPB rows.
// WIDE: 16-byte lanes for every type (8 bfloat16 columns per lane), for
// products with one value set, where a lane may span two subsystems.
template <typename T, int C, bool WIDE = false>
struct Lanes {
    static constexpr int LW = WIDE ? 16 / (int)sizeof(T) : lane_width((int)sizeof(T));
    static constexpr int VW = LW < C ? LW : C;
    static constexpr int LPR = C / VW;
    static constexpr int RPB = kBlock / LPR;
};

// acc[e] += sum over k = k0, k0+step, ... < k1 of va[k] * X[ci[k], lane*VW + e],
// accumulated in that order with four entries' loads in flight at a time.
// With SETS the matrix carries vs interleaved value sets (value of entry k at
// va[k * vs], va offset to the set used).
template <typename T, int C, int VW, typename TV = T, bool SETS = false>
__device__ __forceinline__ void row_accumulate(int32_t k0, int32_t k1, int step, const int32_t* __restrict__ ci,
                                               const TV* __restrict__ va, const T* __restrict__ X, int lane,
                                               acc_t<T>* acc, int vs = 1) {
    using TC = acc_t<T>;
    auto val = [&](int32_t k) -> TC { return cvt<TC>(va[SETS ? (int64_t)k * vs : (int64_t)k]); };
    int32_t k = k0;
    for (; k + 3 * step < k1; k += 4 * step) {
        const int32_t c0 = ci[k], c1 = ci[k + step], c2 = ci[k + 2 * step], c3 = ci[k + 3 * step];
        const TC a0 = val(k), a1 = val(k + step), a2 = val(k + 2 * step), a3 = val(k + 3 * step);
        const Pack<T, VW> x0 = ld<T, VW>(X + (int64_t)c0 * C + lane * VW);
        const Pack<T, VW> x1 = ld<T, VW>(X + (int64_t)c1 * C + lane * VW);
        const Pack<T, VW> x2 = ld<T, VW>(X + (int64_t)c2 * C + lane * VW);
        const Pack<T, VW> x3 = ld<T, VW>(X + (int64_t)c3 * C + lane * VW);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            acc[e] += a0 * to_acc(x0.e[e]);
            acc[e] += a1 * to_acc(x1.e[e]);
            acc[e] += a2 * to_acc(x2.e[e]);
            acc[e] += a3 * to_acc(x3.e[e]);
        }
    }
    for (; k < k1; k += step) {
        const Pack<T, VW> x = ld<T, VW>(X + (int64_t)ci[k] * C + lane * VW);
        const TC a = val(k);
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] += a * to_acc(x.e[e]);
    }
}

// The same sum for rows handled by LPR >= 4 lanes that sit in one wavefront:
// the row's entries are fetched CH = min(LPR, 8) at a time, lane q of the row
// loading entry q (one coalesced load of column indices and values instead of
// every lane reading each entry), and are broadcast with cross-lane shuffles,
// so the CH gathers of X rows are issued back to back.  Entries are added in
// increasing k, the order of row_accumulate.  base = first lane of the row
// within its wavefront.  Every lane of the row must make the call (the
// shuffles read the other lanes' registers).
template <typename T, int C, int VW, int LPR, typename TV = T>
__device__ __forceinline__ void row_accumulate_bcast(int32_t k0, int32_t k1, const int32_t* __restrict__ ci,
                                                     const TV* __restrict__ va, const T* __restrict__ X, int lane,
                                                     int base, acc_t<T>* acc) {
    using TC = acc_t<T>;
    constexpr int CH = LPR < 8 ? LPR : 8;
    for (int32_t kb = k0; kb < k1; kb += CH) {
        const int32_t kk = kb + lane;
        const bool have = lane < CH && kk < k1;
        const int32_t c = have ? ci[kk] : 0;
        const TC a = have ? cvt<TC>(va[kk]) : TC(0);
        const int cnt = k1 - kb < CH ? k1 - kb : CH;
        Pack<T, VW> xs[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int32_t cq = __shfl(c, base + q, 64);
            if (q < cnt) xs[q] = ld<T, VW>(X + (int64_t)cq * C + lane * VW);
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const TC aq = __shfl(a, base + q, 64);
            if (q < cnt) {
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[e] += aq * to_acc(xs[q].e[e]);
            }
        }
    }
}

// The broadcast form for matrices with vs interleaved value sets: only the
// column indices are broadcast; each lane reads the values of its own
// columns' sets (set[e] for column e, from column_sets; one load per entry
// when all VW columns share a set).  Every lane of the row must make the call.
template <typename T, int C, int VW, int LPR, typename TV = T>
__device__ __forceinline__ void row_accumulate_bcast_sets(int32_t k0, int32_t k1, const int32_t* __restrict__ ci,
                                                          const TV* __restrict__ va, const T* __restrict__ X,
                                                          int lane, int base, acc_t<T>* acc, int vs, const int* set,
                                                          bool uniform) {
    using TC = acc_t<T>;
    constexpr int CH = LPR < 8 ? LPR : 8;
    for (int32_t kb = k0; kb < k1; kb += CH) {
        const int32_t kk = kb + lane;
        const bool have = lane < CH && kk < k1;
        const int32_t c = have ? ci[kk] : 0;
        const int cnt = k1 - kb < CH ? k1 - kb : CH;
        Pack<T, VW> xs[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int32_t cq = __shfl(c, base + q, 64);
            if (q < cnt) xs[q] = ld<T, VW>(X + (int64_t)cq * C + lane * VW);
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            if (q < cnt) {
                const TV* vk = va + (int64_t)(kb + q) * vs;
                if (uniform) {
                    const TC a = cvt<TC>(vk[set[0]]);
#pragma unroll
                    for (int e = 0; e < VW; ++e) acc[e] += a * to_acc(xs[q].e[e]);
                } else {
#pragma unroll
                    for (int e = 0; e < VW; ++e) acc[e] += cvt<TC>(vk[set[e]]) * to_acc(xs[q].e[e]);
                }
            }
        }
    }
}

// As row_accumulate with interleaved value sets where the VW columns of the
// lane belong to different sets: column e uses va[k * vs + set[e]].
template <typename T, int C, int VW, typename TV = T>
__device__ __forceinline__ void row_accumulate_sets(int32_t k0, int32_t k1, int step,
                                                    const int32_t* __restrict__ ci, const TV* __restrict__ va,
                                                    const T* __restrict__ X, int lane, acc_t<T>* acc, int vs,
                                                    const int* set) {
    using TC = acc_t<T>;
    for (int32_t k = k0; k < k1; k += step) {
        const Pack<T, VW> x = ld<T, VW>(X + (int64_t)ci[k] * C + lane * VW);
        const TV* vk = va + (int64_t)k * vs;
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] += cvt<TC>(vk[set[e]]) * to_acc(x.e[e]);
    }
}

// Multivector column -> value set: column c belongs to set c / vm (sets own vm
// consecutive columns); padded columns use the last set.
template <int VW>
__device__ __forceinline__ bool column_sets(int lane, int vs, int vm, int* set) {
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        const int q = (lane * VW + e) / vm;
        set[e] = q < vs ? q : vs - 1;
    }
    return set[0] == set[VW - 1];   // sets are nondecreasing in e
}

// Gates of the batched solve.  A batch runs every system's kernels inside one
// captured graph for as many iterations as the slowest system needs; a kernel
// of a system that has no active column left (or has broken down) returns at
// once.  gate: that system's per-column active flags (64 ints, zero past its
// columns), its breakdown flag at gate[128]; nullptr = always run.  The
// decision is a wavefront vote, so every lane of the wavefront must make the
// call, before any lane leaves.
__device__ __forceinline__ bool gate_closed(const int* __restrict__ gate) {
    if (!gate) return false;
    const bool on = gate[threadIdx.x & 63] != 0;
    return gate[128] != 0 || __ballot(on) == 0;
}

// The p update's gate: every column's step alpha is zero (the alpha kernel
// zeroes it on inactive columns), so there is nothing to apply.
__device__ __forceinline__ bool alpha_gate_closed(const double* __restrict__ alpha, bool gated) {
    if (!gated) return false;
    return __ballot(alpha[threadIdx.x & 63] != 0.0) == 0;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Remap so that every XCD works on one contiguous range of logical
// tiles: neighbouring rows, and the multivector rows they gather, then stay
// in the same XCD's L2.  A bijection of [0, nb).
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb) {
    constexpr unsigned X = 8;
    const unsigned q = nb / X, r = nb % X;
    const unsigned x = b % X, i = b / X;
    return x * q + (x < r ? x : r) + i;
}

static inline unsigned blocks_for(int64_t work, int per_block) {
    return (unsigned)((work + per_block - 1) / per_block);
}

// Sum per-thread column partials (VW columns per lane) over the row slots of
// the block in a fixed order; thread c < C writes the block total of column c
// to out[c].  sm must hold kBlock * VW doubles.  Contains __syncthreads().
template <int C, int VW>
__device__ __forceinline__ void block_column_sums(const double* acc, double* sm, double* out) {
    constexpr int LPR = C / VW;
    constexpr int RPB = kBlock / LPR;
#pragma unroll
    for (int e = 0; e < VW; ++e) sm[threadIdx.x * VW + e] = acc[e];
    __syncthreads();
    if (threadIdx.x < C) {
        double s = 0.0;
        for (int r = 0; r < RPB; ++r) s += sm[r * C + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Tree sum of partial[b * O + o] over b < nb for one output o per block
// (fixed order); result valid in thread 0.
__device__ __forceinline__ double block_sum_partials(int nb, int O, int o, const double* partial, double* sm) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) s += partial[(int64_t)b * O + o];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (unsigned w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    return sm[0];
}

}  // namespace msp
