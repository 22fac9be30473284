// Sliced-ELL SpMM for the V-cycle products (gfx950, wave64).
//
// Format (built on the host from the CSR of a V-cycle matrix, build_sell in api.cpp):
// every row is split into G virtual rows (virtual row v = row * G + g holds
// the row's entries j = g, g + G, g + 2G, ... in their CSR order), and the
// virtual rows are cut into slices of 64.  Slice s has a width wid[s] (the
// longest virtual row in it) and its entries are stored column-major from slot
// off[s]: entry k of virtual row v sits in slot off[s] + 64 k + (v mod 64),
// with column -1 (and value 0) in padding slots.  Values carry vs interleaved
// value sets like the CSR form (slot q of set a at va[q * vs + a]).
//
// A wavefront covers 64 / LPR consecutive virtual rows of one slice (LPR
// lanes per row, VW columns per lane, as in the CSR kernels).  The slice's
// width and offset are the same for the whole wavefront, so the loop over k
// runs without a row-pointer load: each step issues the column indices and
// values of 8 entries (one coalesced load per entry for the wavefront), then
// their 8 gathers of X rows, so a product needs two dependent memory steps
// per 8 entries instead of three.  The G partial sums of a row sit in lanes
// LPR apart inside one wavefront and are added by a fixed butterfly of
// cross-lane shuffles; the row's first group writes Y.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace msp {

constexpr int kSellH = 64;   // virtual rows per slice
constexpr int kSellU = 8;    // entries whose loads are in flight together

template <typename T, typename TV, int C, int G, bool SETS, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_sell(int64_t n, const int64_t* __restrict__ off,
                                                 const int32_t* __restrict__ wid, const int32_t* __restrict__ ci,
                                                 const TV* __restrict__ va, const T* __restrict__ X, T* Y, const T* Z,
                                                 acc_t<T> alpha, acc_t<T> beta, OuterDiag sigma, int S, int m,
                                                 int vs, const int* __restrict__ gate) {
    if (gate_closed(gate)) return;
    using L = Lanes<T, C, WIDE>;
    using TC = acc_t<T>;
    constexpr int VW = L::VW, LPR = L::LPR;
    constexpr int VPW = 64 / LPR;        // virtual rows per wavefront
    constexpr int VPB = kBlock / LPR;    // virtual rows per block
    static_assert(G * LPR <= 64, "the lanes of one row must sit in one wavefront");
    static_assert(kSellH % VPW == 0, "a wavefront's rows must sit in one slice");
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t nv = n * G;
    const int64_t v = tile * VPB + threadIdx.x / LPR;
    const int lane = threadIdx.x % LPR;
    const int64_t row = v / G;
    const int g = (int)(v % G);
    const bool live = v < nv;
    const bool out = live && g == 0;
    // first virtual row of this wavefront (the same for all its lanes)
    const int64_t v0 = tile * VPB + (int64_t)(threadIdx.x / 64) * VPW;
    int w = 0;
    int64_t slot = 0;
    if (v0 < nv) {
        const int64_t s = v0 / kSellH;
        w = __builtin_amdgcn_readfirstlane(wid[s]);
        slot = off[s] + (v % kSellH);
    }
    Pack<T, VW> zv{};
    if (Z && out) zv = ld<T, VW>(Z + row * C + lane * VW);
    TC acc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = TC(0);
    int set[VW] = {};
    bool uniform = true;
    if constexpr (SETS) uniform = column_sets<VW>(lane, vs, m, set);
    const int vo = SETS ? set[0] : 0;   // value-set offset when the lane's columns share one set
    for (int k0 = 0; k0 < w; k0 += kSellU) {
        // column indices and (one set per lane) values of kSellU entries, then their gathers
        int32_t cc[kSellU];
        TC aa[kSellU];
#pragma unroll
        for (int u = 0; u < kSellU; ++u) {
            const int64_t q = slot + (int64_t)(k0 + u) * kSellH;
            const bool in = live && k0 + u < w;
            cc[u] = in ? ci[q] : -1;
            aa[u] = (in && uniform) ? cvt<TC>(va[q * vs + vo]) : TC(0);
        }
        Pack<T, VW> xs[kSellU];
#pragma unroll
        for (int u = 0; u < kSellU; ++u) {
            if (cc[u] >= 0) {
                xs[u] = ld<T, VW>(X + (int64_t)cc[u] * C + lane * VW);
            } else {
#pragma unroll
                for (int e = 0; e < VW; ++e) xs[u].e[e] = T{};
            }
        }
#pragma unroll
        for (int u = 0; u < kSellU; ++u) {
            if (cc[u] < 0) continue;
            if (uniform) {
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[e] += aa[u] * to_acc(xs[u].e[e]);
            } else {   // the lane's columns belong to several value sets
                const int64_t q = slot + (int64_t)(k0 + u) * kSellH;
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[e] += cvt<TC>(va[q * vs + set[e]]) * to_acc(xs[u].e[e]);
            }
        }
    }
    // the G partial sums of a row: lanes g * LPR + lane of its 64-lane-aligned group
#pragma unroll
    for (int o = LPR; o < G * LPR; o <<= 1)
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] += __shfl_xor(acc[e], o, 64);
    if (!out) return;
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
    Pack<T, VW> res;
    if (Z) {
#pragma unroll
        for (int e = 0; e < VW; ++e) res.e[e] = from_acc<T>(alpha * acc[e] + beta * to_acc(zv.e[e]));
    } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) res.e[e] = from_acc<T>(alpha * acc[e]);
    }
    st<T, VW>(Y + row * C + lane * VW, res);
}

// ------------------------------------------------------------------ launcher

template <typename T, typename TV, int CC, int G>
static void sell_launch_g(hipStream_t st, int64_t n, const int64_t* off, const int32_t* wid, const int32_t* ci,
                          const TV* va, const T* X, T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta,
                          OuterDiag sigma, int S, int m, int vs, bool wide, const int* gate) {
    using LN = Lanes<T, CC, false>;
    using LW = Lanes<T, CC, true>;
    const bool w = wide && vs == 1 && LW::VW != LN::VW;
    if constexpr (G * LW::LPR <= 64) {
        if (w) {
            constexpr int VPB = kBlock / LW::LPR;
            hipLaunchKernelGGL((k_sell<T, TV, CC, G, false, true>), dim3(blocks_for(n * G, VPB)), dim3(kBlock), 0, st,
                               n, off, wid, ci, va, X, Y, Z, alpha, beta, sigma, S, m, 1, gate);
            return;
        }
    }
    if constexpr (G * LN::LPR <= 64) {
        constexpr int VPB = kBlock / LN::LPR;
        if (vs > 1)
            hipLaunchKernelGGL((k_sell<T, TV, CC, G, true, false>), dim3(blocks_for(n * G, VPB)), dim3(kBlock), 0, st,
                               n, off, wid, ci, va, X, Y, Z, alpha, beta, sigma, S, m, vs, gate);
        else
            hipLaunchKernelGGL((k_sell<T, TV, CC, G, false, false>), dim3(blocks_for(n * G, VPB)), dim3(kBlock), 0,
                               st, n, off, wid, ci, va, X, Y, Z, alpha, beta, sigma, S, m, 1, gate);
    }
}

bool sell_fits(int C, int elem_bytes, int G, bool wide) {
    const int lw = wide ? 16 / elem_bytes : lane_width(elem_bytes);
    const int vw = lw < C ? lw : C;
    return G >= 1 && G * (C / vw) <= 64;
}

template <typename T, typename TV>
hipError_t launch_sell(hipStream_t st, int C, int G, int64_t n, const int64_t* off, const int32_t* wid,
                       const int32_t* ci, const TV* va, const T* X, T* Y, const T* Z, acc_t<T> alpha, acc_t<T> beta,
                       OuterDiag sigma, int S, int m, int vs, bool wide, const int* gate) {
    if (n <= 0) return hipSuccess;
    if ((vs > 1 || sigma.idx) && m < 1) return hipErrorInvalidValue;
    if (!sell_fits(C, (int)sizeof(T), G, wide && vs == 1)) return hipErrorInvalidValue;
#define MSP_SELL_G(CC)                                                                                         \
    switch (G) {                                                                                               \
        case 1: sell_launch_g<T, TV, CC, 1>(st, n, off, wid, ci, va, X, Y, Z, alpha, beta, sigma, S, m, vs,   \
                                            wide, gate);                                                       \
            break;                                                                                             \
        case 2: sell_launch_g<T, TV, CC, 2>(st, n, off, wid, ci, va, X, Y, Z, alpha, beta, sigma, S, m, vs,   \
                                            wide, gate);                                                       \
            break;                                                                                             \
        case 4: sell_launch_g<T, TV, CC, 4>(st, n, off, wid, ci, va, X, Y, Z, alpha, beta, sigma, S, m, vs,   \
                                            wide, gate);                                                       \
            break;                                                                                             \
        case 8: sell_launch_g<T, TV, CC, 8>(st, n, off, wid, ci, va, X, Y, Z, alpha, beta, sigma, S, m, vs,   \
                                            wide, gate);                                                       \
            break;                                                                                             \
        case 16: sell_launch_g<T, TV, CC, 16>(st, n, off, wid, ci, va, X, Y, Z, alpha, beta, sigma, S, m, vs, \
                                              wide, gate);                                                     \
            break;                                                                                             \
        default: return hipErrorInvalidValue;                                                                  \
    }
    switch (C) {
        case 1: MSP_SELL_G(1) break;
        case 2: MSP_SELL_G(2) break;
        case 4: MSP_SELL_G(4) break;
        case 8: MSP_SELL_G(8) break;
        case 16: MSP_SELL_G(16) break;
        case 32: MSP_SELL_G(32) break;
        case 64: MSP_SELL_G(64) break;
        default: return hipErrorInvalidValue;
    }
#undef MSP_SELL_G
    return hipGetLastError();
}

#define MSP_SELL_INST(T, TV)                                                                                      \
    template hipError_t launch_sell<T, TV>(hipStream_t, int, int, int64_t, const int64_t*, const int32_t*,       \
                                           const int32_t*, const TV*, const T*, T*, const T*, acc_t<T>, acc_t<T>, \
                                           OuterDiag, int, int, int, bool, const int*);
MSP_SELL_INST(double, double)
MSP_SELL_INST(float, float)
MSP_SELL_INST(Bf16, float)

}  // namespace msp
