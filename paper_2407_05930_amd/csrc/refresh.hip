// Kernels of the numeric re-setup on the device: every value of the hierarchy
// recomputed for a new matrix on the structure (C/F splits, patterns) of an
// earlier setup.  One thread per row replays the host setup's arithmetic in
// the same order (contraction off), so a re-setup with the setup's own matrix
// reproduces the host values to rounding.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "refresh.hpp"

#pragma clang fp contract(off)

namespace msp {

namespace {

constexpr int kRB = 256;

__device__ __forceinline__ int64_t find_col(const int32_t* __restrict__ ci, int64_t b, int64_t e, int32_t q) {
    while (b < e) {
        const int64_t m = (b + e) >> 1;
        const int32_t v = ci[m];
        if (v < q) b = m + 1;
        else if (v > q) e = m;
        else return m;
    }
    return -1;
}

__device__ __forceinline__ double lookup(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                         const double* __restrict__ v, int32_t i, int32_t j) {
    const int64_t p = find_col(ci, rp[i], rp[i + 1], j);
    return p >= 0 ? v[p] : 0.0;
}

unsigned grid_for(int64_t n) {
    const int64_t b = (n + kRB - 1) / kRB;
    return static_cast<unsigned>(b < 1 ? 1 : (b > 65535 * 16 ? 65535 * 16 : b));
}

__global__ __launch_bounds__(kRB) void k_gather(int64_t n, const int64_t* __restrict__ src,
                                                const double* __restrict__ in, double* __restrict__ out, int stride,
                                                int offset) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRB) {
        const int64_t s = src[i];
        out[i * stride + offset] = s >= 0 ? in[s] : 0.0;
    }
}

__global__ __launch_bounds__(kRB) void k_strided_copy(int64_t n, const double* __restrict__ in, int istride,
                                                      int ioff, double* __restrict__ out, int ostride, int ooff) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRB)
        out[i * ostride + ooff] = in[i * istride + ioff];
}

// sigma[i*S + a] = sum_{j=1..S-1} (-1)^{popcount(a & j)} h_j(i), h_j from the
// caller's values (src = -1: no such coupling), summed in increasing j.
__global__ __launch_bounds__(kRB) void k_outer_sigma(int64_t nb, int S, const int64_t* __restrict__ src,
                                                     const double* __restrict__ val, double* __restrict__ sigma) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (i >= nb) return;
    double h[64];
    h[0] = 0.0;
    for (int j = 1; j < S; ++j) {
        const int64_t s = src[i * (S - 1) + (j - 1)];
        h[j] = s >= 0 ? val[s] : 0.0;
    }
    for (int a = 0; a < S; ++a) {
        double acc = 0.0;
        for (int j = 1; j < S; ++j) {
            const double t = (__popc(static_cast<unsigned>(a & j)) & 1) ? -h[j] : h[j];
            acc = acc + t;
        }
        sigma[i * S + a] = acc;
    }
}

// A_1,a = A_1 + sigma_a on the interface's coarse points: v[diag[q]] += sigma[base[q]*S + a]
__global__ __launch_bounds__(kRB) void k_add_sigma(int64_t nq, const int64_t* __restrict__ diag,
                                                   const int64_t* __restrict__ base, const double* __restrict__ sigma,
                                                   int S, int a, double* __restrict__ v) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (q >= nq) return;
    double& d = v[diag[q]];
    d = d + sigma[base[q] * S + a];
}

// One Jacobi step of the interpolation for F row r (fine row fidx[r]):
// W_new = -D^{-1} (A_FC + O W_prev) on W_new's symbolic pattern.
__global__ __launch_bounds__(kRB) void k_interp_step(int64_t nf, const int32_t* __restrict__ fidx,
                                                     const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                                     const double* __restrict__ av, const int8_t* __restrict__ cf,
                                                     const int32_t* __restrict__ cnum, const int32_t* __restrict__ fnum,
                                                     const int32_t* __restrict__ prp, const int32_t* __restrict__ pci,
                                                     const double* __restrict__ pv, const int32_t* __restrict__ wrp,
                                                     const int32_t* __restrict__ wci, double* __restrict__ wv,
                                                     double* __restrict__ afc, int8_t* __restrict__ hasf,
                                                     int* __restrict__ err) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (r >= nf) return;
    const int32_t i = fidx[r];
    const int64_t wb = wrp[r], we = wrp[r + 1];
    for (int64_t p = wb; p < we; ++p) {
        wv[p] = 0.0;
        afc[p] = 0.0;
        hasf[p] = 0;
    }
    double dii = 0.0;
    for (int64_t k = arp[i]; k < arp[i + 1]; ++k) {
        const int32_t c = aci[k];
        if (c == i) {
            dii = av[k];
            continue;
        }
        if (cf[c]) {
            const int64_t p = find_col(wci, wb, we, cnum[c]);
            if (p < 0) {
                atomicOr(err, 1);
                continue;
            }
            afc[p] = av[k];
            hasf[p] = 1;
        } else if (prp) {
            const int32_t f = fnum[c];
            const double a = av[k];
            for (int64_t q = prp[f]; q < prp[f + 1]; ++q) {
                const int64_t p = find_col(wci, wb, we, pci[q]);
                if (p < 0) {
                    atomicOr(err, 1);
                    continue;
                }
                wv[p] += a * pv[q];
            }
        }
    }
    const double dinv = 1.0 / dii;
    for (int64_t p = wb; p < we; ++p) {
        const double t = hasf[p] ? afc[p] + wv[p] : wv[p];
        wv[p] = -(dinv * t);
    }
}

// P row i: the unit row of a C point, or the kept weights of an F point
// (pmap: P entry -> entry of the last Jacobi step) rescaled to the row sum
// rho_i = -sum_{l != i} a_il / a_ii.
__global__ __launch_bounds__(kRB) void k_interp_finish(int64_t n, const int8_t* __restrict__ cf,
                                                       const int32_t* __restrict__ arp,
                                                       const int32_t* __restrict__ aci,
                                                       const double* __restrict__ av, const double* __restrict__ wv,
                                                       const int32_t* __restrict__ prp,
                                                       const int32_t* __restrict__ pmap, double* __restrict__ pv) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (i >= n) return;
    const int64_t pb = prp[i], pe = prp[i + 1];
    if (cf[i]) {
        pv[pb] = 1.0;
        return;
    }
    double off = 0.0, dii = 0.0;
    for (int64_t k = arp[i]; k < arp[i + 1]; ++k) {
        if (aci[k] == i) dii = av[k];
        else off += av[k];
    }
    const double rho = -off / dii;
    double ws = 0.0;
    for (int64_t e = pb; e < pe; ++e) ws += wv[pmap[e]];
    if (ws != 0.0) {
        const double sc = rho / ws;
        for (int64_t e = pb; e < pe; ++e) pv[e] = wv[pmap[e]] * sc;
    } else {
        for (int64_t e = pb; e < pe; ++e) pv[e] = wv[pmap[e]];
    }
}

// Static FSAI row i on G's pattern J (last entry i): A[J,J] = L L^T,
// L L^T g = e_last, row = g / sqrt(g_last).  work + woff[i] holds k*k + k doubles.
__global__ __launch_bounds__(kRB) void k_fsai(int64_t n, const int32_t* __restrict__ arp,
                                              const int32_t* __restrict__ aci, const double* __restrict__ av,
                                              const int32_t* __restrict__ grp, const int32_t* __restrict__ gci,
                                              double* __restrict__ gv, const int64_t* __restrict__ woff,
                                              double* __restrict__ work, int* __restrict__ err) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (i >= n) return;
    const int64_t gb = grp[i];
    const int k = static_cast<int>(grp[i + 1] - gb);
    const int32_t* J = gci + gb;
    double* M = work + woff[i];
    double* g = M + static_cast<int64_t>(k) * k;
    for (int p = 0; p < k; ++p)
        for (int q = 0; q < k; ++q) M[p * k + q] = lookup(arp, aci, av, J[p], J[q]);
    for (int j = 0; j < k; ++j) {   // Cholesky, lower factor in place
        double d = M[j * k + j];
        for (int p = 0; p < j; ++p) d -= M[j * k + p] * M[j * k + p];
        if (!(d > 0.0)) {
            atomicOr(err, 2);
            return;
        }
        d = sqrt(d);
        M[j * k + j] = d;
        for (int r = j + 1; r < k; ++r) {
            double s = M[r * k + j];
            for (int p = 0; p < j; ++p) s -= M[r * k + p] * M[j * k + p];
            M[r * k + j] = s / d;
        }
    }
    for (int p = 0; p < k; ++p) g[p] = 0.0;
    g[k - 1] = 1.0 / M[(k - 1) * k + (k - 1)];
    for (int p = k - 1; p >= 0; --p) {
        double s = g[p];
        for (int q = p + 1; q < k; ++q) s -= M[q * k + p] * g[q];
        g[p] = s / M[p * k + p];
    }
    const double sc = 1.0 / sqrt(g[k - 1]);
    for (int p = 0; p < k; ++p) gv[gb + p] = g[p] * sc;
}

// C = A B on C's kept pattern, one thread per nonzero of C: entry (i, c) sums
// a_ik b_kc over the row of A in its order (the order in which a row-wise
// product accumulates it), b_kc found by binary search in row k of B.  The
// kept pattern is the symbolic product of the kept patterns, so every
// product term has its slot.
__global__ __launch_bounds__(kRB) void k_spgemm_masked(int64_t nr, int64_t nnz, const int32_t* __restrict__ arp,
                                                       const int32_t* __restrict__ aci,
                                                       const double* __restrict__ av,
                                                       const int32_t* __restrict__ brp,
                                                       const int32_t* __restrict__ bci,
                                                       const double* __restrict__ bv,
                                                       const int32_t* __restrict__ crp,
                                                       const int32_t* __restrict__ cci, double* __restrict__ cv) {
    for (int64_t p = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; p < nnz;
         p += static_cast<int64_t>(gridDim.x) * kRB) {
        int64_t lo = 0, hi = nr;   // the row i with crp[i] <= p < crp[i + 1]
        while (hi - lo > 1) {
            const int64_t m = (lo + hi) >> 1;
            if (crp[m] <= p) lo = m;
            else hi = m;
        }
        const int32_t c = cci[p];
        double s = 0.0;
        for (int64_t k = arp[lo]; k < arp[lo + 1]; ++k) {
            const int32_t j = aci[k];
            const int64_t q = find_col(bci, brp[j], brp[j + 1], c);
            if (q >= 0) s += av[k] * bv[q];
        }
        cv[p] = s;
    }
}

// Split of the reduction level that a fresh setup would take (Alg. 2): the
// strength of connection marks entry (i, j), j != i, when -a_ij >= theta * max_{l != i}(-a_il) (no entry
// when that maximum is <= 0); T is its symmetric closure.
__global__ __launch_bounds__(kRB) void k_strength(int64_t n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                  double theta, int8_t* __restrict__ smask) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRB) {
        double mx = -INFINITY;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] != i) mx = fmax(mx, -v[k]);
        const double thr = theta * mx;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            smask[k] = (mx > 0.0 && ci[k] != i && -v[k] >= thr) ? 1 : 0;
    }
}

__global__ __launch_bounds__(kRB) void k_symmetric_mask(int64_t nnz, const int64_t* __restrict__ tmap,
                                                        const int8_t* __restrict__ smask,
                                                        int8_t* __restrict__ tmask) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; k < nnz;
         k += static_cast<int64_t>(gridDim.x) * kRB)
        tmask[k] = (smask[k] | smask[tmap[k]]) ? 1 : 0;
}

constexpr int8_t kUndecided = 0, kIn = 1, kOut = 2, kNotCandidate = 3;

// Does a node y within d <= 3 hops of u (through candidates, along T) satisfy
// pred(y)?  u itself is not visited.
template <typename Pred>
__device__ bool any_within(int64_t u, int d, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const int8_t* __restrict__ tmask, const int8_t* __restrict__ state, Pred pred) {
    for (int64_t k1 = rp[u]; k1 < rp[u + 1]; ++k1) {
        if (!tmask[k1]) continue;
        const int32_t y1 = ci[k1];
        if (state[y1] == kNotCandidate) continue;
        if (y1 != u && pred(y1)) return true;
        if (d < 2) continue;
        for (int64_t k2 = rp[y1]; k2 < rp[y1 + 1]; ++k2) {
            if (!tmask[k2]) continue;
            const int32_t y2 = ci[k2];
            if (y2 == u || state[y2] == kNotCandidate) continue;
            if (pred(y2)) return true;
            if (d < 3) continue;
            for (int64_t k3 = rp[y2]; k3 < rp[y2 + 1]; ++k3) {
                if (!tmask[k3]) continue;
                const int32_t y3 = ci[k3];
                if (y3 == u || state[y3] == kNotCandidate) continue;
                if (pred(y3)) return true;
            }
        }
    }
    return false;
}

// One round: an undecided candidate joins when no candidate within d hops
// that is not out has a higher priority (writing "in" in place is harmless:
// in and undecided both count as not out).  Priority: lam first (when given,
// the number of strong dependants), then pri.
__global__ __launch_bounds__(kRB) void k_mis_select(int64_t n, int d, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const int8_t* __restrict__ tmask,
                                                    const int32_t* __restrict__ lam, const uint64_t* __restrict__ pri,
                                                    int8_t* __restrict__ state) {
    for (int64_t u = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * kRB) {
        if (state[u] != kUndecided) continue;
        const uint64_t pu = pri[u];
        const int32_t lu = lam ? lam[u] : 0;
        const bool beaten = any_within(u, d, rp, ci, tmask, state, [&](int32_t y) {
            if (state[y] == kOut) return false;
            const int32_t ly = lam ? lam[y] : 0;
            return ly > lu || (ly == lu && pri[y] > pu);
        });
        if (!beaten) state[u] = kIn;
    }
}

// lam[i] = number of rows j whose strong set holds i
__global__ __launch_bounds__(kRB) void k_strong_dependants(int64_t n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const int8_t* __restrict__ smask,
                                                           int32_t* __restrict__ lam) {
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * kRB)
        for (int64_t k = rp[j]; k < rp[j + 1]; ++k)
            if (smask[k]) atomicAdd(&lam[ci[k]], 1);
}

// Undecided candidates with a member within d hops leave; counts the rest.
__global__ __launch_bounds__(kRB) void k_mis_remove(int64_t n, int d, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const int8_t* __restrict__ tmask,
                                                    int8_t* __restrict__ state, int* __restrict__ left) {
    for (int64_t u = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * kRB) {
        if (state[u] != kUndecided) continue;
        if (any_within(u, d, rp, ci, tmask, state, [&](int32_t y) { return state[y] == kIn; })) state[u] = kOut;
        else atomicAdd(left, 1);
    }
}

// number of points whose decision (C: member or not a candidate) differs from cf
__global__ __launch_bounds__(kRB) void k_split_diff(int64_t n, const int8_t* __restrict__ state,
                                                    const int8_t* __restrict__ cf,
                                                    unsigned long long* __restrict__ count) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRB) {
        const int8_t c = (state[i] == kIn || state[i] == kNotCandidate) ? 1 : 0;
        if (c != (cf[i] ? 1 : 0)) atomicAdd(count, 1ull);
    }
}

// one wavefront per row (rows with many entries); lanes stride over the row,
// then a butterfly sum
__global__ __launch_bounds__(kRB) void k_spmv_wave(int64_t n, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                   const double* __restrict__ x, double* __restrict__ y) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * (kRB / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (i >= n) return;   // the whole wavefront leaves together
    double s = 0.0;
    for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += 64) s += v[k] * x[ci[k]];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) y[i] = s;
}

// values of a sliced-ELL form from its CSR values: slot q of set a holds entry
// pos[q] of set a (pos < 0: padding, zero)
__global__ __launch_bounds__(kRB) void k_sell_values(int64_t slots, int vs, const int64_t* __restrict__ pos,
                                                     const double* __restrict__ v, double* __restrict__ out64,
                                                     float* __restrict__ out32) {
    const int64_t total = slots * vs;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * kRB) {
        const int64_t q = t / vs, a = t - q * vs;
        const int64_t p = pos[q];
        const double x = p >= 0 ? v[p * vs + a] : 0.0;
        if (out32) out32[t] = static_cast<float>(x);
        else out64[t] = x;
    }
}

// Energy minimisation of an interpolation P (n rows, C rows unit rows), one
// thread per row.  Projection onto the row-sum constraint: on F rows v minus
// its row mean (times sign), C rows zero.
__global__ __launch_bounds__(kRB) void k_emin_project(int64_t n, const int32_t* __restrict__ rp,
                                                      const int8_t* __restrict__ cf, const double* __restrict__ v,
                                                      double sign, double* __restrict__ out) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRB) {
        const int64_t b = rp[i], e = rp[i + 1];
        if (cf[i]) {
            for (int64_t k = b; k < e; ++k) out[k] = 0.0;
            continue;
        }
        double s = 0.0;
        for (int64_t k = b; k < e; ++k) s += v[k];
        const double mean = e > b ? s / static_cast<double>(e - b) : 0.0;
        for (int64_t k = b; k < e; ++k) out[k] = sign * (v[k] - mean);
    }
}

// dinv[k] = 1 / a_ii for every entry k of row i of P
__global__ __launch_bounds__(kRB) void k_emin_dinv(int64_t n, const int32_t* __restrict__ arp,
                                                   const int32_t* __restrict__ aci, const double* __restrict__ av,
                                                   const int32_t* __restrict__ prp, double* __restrict__ dinv) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRB) {
        const double d = 1.0 / lookup(arp, aci, av, static_cast<int32_t>(i), static_cast<int32_t>(i));
        for (int64_t k = prp[i]; k < prp[i + 1]; ++k) dinv[k] = d;
    }
}

// w += alpha p, r -= alpha q, z = dinv r
__global__ __launch_bounds__(kRB) void k_emin_step(int64_t m, double alpha, const double* __restrict__ p,
                                                   const double* __restrict__ q, const double* __restrict__ dinv,
                                                   double* __restrict__ w, double* __restrict__ r,
                                                   double* __restrict__ z) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; k < m;
         k += static_cast<int64_t>(gridDim.x) * kRB) {
        w[k] = w[k] + alpha * p[k];
        const double rn = r[k] - alpha * q[k];
        r[k] = rn;
        z[k] = dinv[k] * rn;
    }
}

// p = z + beta p (beta = 0: p = z)
__global__ __launch_bounds__(kRB) void k_emin_dir(int64_t m, double beta, const double* __restrict__ z,
                                                  double* __restrict__ p) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; k < m;
         k += static_cast<int64_t>(gridDim.x) * kRB)
        p[k] = z[k] + beta * p[k];
}

__global__ __launch_bounds__(kRB) void k_mul(int64_t m, const double* __restrict__ a, const double* __restrict__ b,
                                             double* __restrict__ out) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; k < m;
         k += static_cast<int64_t>(gridDim.x) * kRB)
        out[k] = a[k] * b[k];
}

__global__ __launch_bounds__(kRB) void k_scale(int64_t n, double* __restrict__ v, double s) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRB)
        v[i] = v[i] * s;
}

__global__ __launch_bounds__(kRB) void k_spmv(int64_t n, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci, const double* __restrict__ v,
                                              const double* __restrict__ x, double* __restrict__ y) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
    y[i] = s;
}

// partial sums of x.y and y.y per block, in a fixed order
__global__ __launch_bounds__(kRB) void k_dots2(int64_t n, const double* __restrict__ x,
                                               const double* __restrict__ y, double* __restrict__ part) {
    __shared__ double sa[kRB], sb[kRB];
    double a = 0.0, b = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRB) {
        a += x[i] * y[i];
        b += y[i] * y[i];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int h = kRB / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) {
            sa[threadIdx.x] += sa[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa[0];
        part[2 * blockIdx.x + 1] = sb[0];
    }
}

// out[0] = sum of the x.y partials, out[1] = sum of the y.y partials (one thread, fixed order)
__global__ void k_dots2_finish(int nb, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int q = 0; q < nb; ++q) {
        a += part[2 * q];
        b += part[2 * q + 1];
    }
    out[0] = a;
    out[1] = b;
}

__global__ __launch_bounds__(kRB) void k_normalise(int64_t n, const double* __restrict__ w,
                                                   const double* __restrict__ dots, double* __restrict__ v) {
    const double wn = sqrt(dots[1]);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRB)
        v[i] = w[i] / wn;
}

// dense n x n row-major copies of S CSR value sets (set a: values at v[k*S + a])
__global__ __launch_bounds__(kRB) void k_densify(int64_t n, int S, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                 double* __restrict__ X) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (t >= n * S) return;
    const int64_t a = t / n, i = t % n;
    double* row = X + (a * n + i) * n;
    for (int64_t j = 0; j < n; ++j) row[j] = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) row[ci[k]] = v[k * S + a];
}

// Gauss-Jordan inversion in place, step k: keep row k and column k of every set
__global__ __launch_bounds__(kRB) void k_gj_keep(int64_t n, int S, int64_t k, const double* __restrict__ X,
                                                 double* __restrict__ rowk, double* __restrict__ colk) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (t >= n * S) return;
    const int64_t a = t / n, j = t % n;
    const double* M = X + a * n * n;
    rowk[a * n + j] = M[k * n + j];
    colk[a * n + j] = M[j * n + k];
}

__global__ __launch_bounds__(kRB) void k_gj_update(int64_t n, int S, int64_t k, double* __restrict__ X,
                                                   const double* __restrict__ rowk,
                                                   const double* __restrict__ colk) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (t >= n * n * S) return;
    const int64_t a = t / (n * n), e = t % (n * n), i = e / n, j = e % n;
    const double p = rowk[a * n + k];
    const double rj = rowk[a * n + j], ci = colk[a * n + i];
    double& x = X[t];
    if (i == k) x = (j == k) ? 1.0 / p : rj / p;
    else x = (j == k) ? -(ci / p) : x - ci * (rj / p);
}

// Two-point-flux transmissibility of face q (interior: harmonic mean of the
// two half-cell conductances; Dirichlet wall; mirror plane at half the
// distance), the host assembly's arithmetic.
__global__ __launch_bounds__(kRB) void k_fv_face_T(int64_t nf, const int64_t* __restrict__ ca,
                                                   const int64_t* __restrict__ cb, const int8_t* __restrict__ kind,
                                                   const double* __restrict__ area, const double* __restrict__ da,
                                                   const double* __restrict__ db, const double* __restrict__ kap,
                                                   double* __restrict__ T) {
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; q < nf;
         q += static_cast<int64_t>(gridDim.x) * kRB) {
        const double ka = kap[ca[q]];
        const int K = kind[q];
        T[q] = K == 0 ? area[q] / (da[q] / ka + db[q] / kap[cb[q]])
                      : (K == 1 ? area[q] * ka / da[q] : area[q] * ka / (2.0 * da[q]));
    }
}

// diagonal of base cell i: the sum of its faces' T in incidence order
__global__ __launch_bounds__(kRB) void k_fv_diag(int64_t nb, const int64_t* __restrict__ cfp,
                                                 const int32_t* __restrict__ cfi, const double* __restrict__ T,
                                                 double* __restrict__ diag) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; i < nb;
         i += static_cast<int64_t>(gridDim.x) * kRB) {
        double s = 0.0;
        for (int64_t e = cfp[i]; e < cfp[i + 1]; ++e) s += T[cfi[e]];
        diag[i] = s;
    }
}

__global__ __launch_bounds__(kRB) void k_fv_values(int64_t nnz, const int32_t* __restrict__ slot,
                                                   const double* __restrict__ T, const double* __restrict__ diag,
                                                   double* __restrict__ val) {
    for (int64_t p = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x; p < nnz;
         p += static_cast<int64_t>(gridDim.x) * kRB) {
        const int32_t c = slot[p];
        val[p] = c >= 0 ? -T[c] : diag[-static_cast<int64_t>(c) - 1];
    }
}

__global__ __launch_bounds__(kRB) void k_dense_to_f32(int64_t rows, int64_t n, int64_t ld,
                                                      const double* __restrict__ X, float* __restrict__ out) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kRB + threadIdx.x;
    if (t >= rows * ld) return;
    const int64_t r = t / ld, k = t % ld;
    out[t] = k < n ? static_cast<float>(X[r * n + k]) : 0.0f;
}

}  // namespace

hipError_t launch_fv_values(hipStream_t st, int64_t nf, int64_t nb, int64_t nnz, const int64_t* ca, const int64_t* cb,
                            const int8_t* kind, const double* area, const double* da, const double* db,
                            const int64_t* cfp, const int32_t* cfi, const int32_t* slot, const double* kap, double* T,
                            double* diag, double* val) {
    if (nf > 0)
        hipLaunchKernelGGL(k_fv_face_T, dim3(grid_for(nf)), dim3(kRB), 0, st, nf, ca, cb, kind, area, da, db, kap, T);
    hipLaunchKernelGGL(k_fv_diag, dim3(grid_for(nb)), dim3(kRB), 0, st, nb, cfp, cfi, T, diag);
    hipLaunchKernelGGL(k_fv_values, dim3(grid_for(nnz)), dim3(kRB), 0, st, nnz, slot, T, diag, val);
    return hipGetLastError();
}

hipError_t launch_dense_to_f32(hipStream_t st, int S, int64_t n, int64_t ld, const double* X, float* out) {
    const int64_t rows = static_cast<int64_t>(S) * n;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dense_to_f32, dim3(static_cast<unsigned>((rows * ld + kRB - 1) / kRB)), dim3(kRB), 0, st,
                       rows, n, ld, X, out);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t st, int64_t n, const int64_t* src, const double* in, double* out, int stride,
                         int offset) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(kRB), 0, st, n, src, in, out, stride, offset);
    return hipGetLastError();
}

hipError_t launch_strided_copy(hipStream_t st, int64_t n, const double* in, int istride, int ioff, double* out,
                               int ostride, int ooff) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_strided_copy, dim3(grid_for(n)), dim3(kRB), 0, st, n, in, istride, ioff, out, ostride, ooff);
    return hipGetLastError();
}

hipError_t launch_outer_sigma(hipStream_t st, int64_t nb, int S, const int64_t* src, const double* val,
                              double* sigma) {
    if (S < 1 || S > 64) return hipErrorInvalidValue;
    if (S == 1) return hipMemsetAsync(sigma, 0, sizeof(double) * nb, st);
    hipLaunchKernelGGL(k_outer_sigma, dim3(static_cast<unsigned>((nb + kRB - 1) / kRB)), dim3(kRB), 0, st, nb, S,
                       src, val, sigma);
    return hipGetLastError();
}

hipError_t launch_add_sigma(hipStream_t st, int64_t nq, const int64_t* diag, const int64_t* base,
                            const double* sigma, int S, int a, double* v) {
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_sigma, dim3(static_cast<unsigned>((nq + kRB - 1) / kRB)), dim3(kRB), 0, st, nq, diag,
                       base, sigma, S, a, v);
    return hipGetLastError();
}

hipError_t launch_interp_step(hipStream_t st, int64_t nf, const int32_t* fidx, const int32_t* arp,
                              const int32_t* aci, const double* av, const int8_t* cf, const int32_t* cnum,
                              const int32_t* fnum, const int32_t* prp, const int32_t* pci, const double* pv,
                              const int32_t* wrp, const int32_t* wci, double* wv, double* afc, int8_t* hasf,
                              int* err) {
    if (nf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_interp_step, dim3(static_cast<unsigned>((nf + kRB - 1) / kRB)), dim3(kRB), 0, st, nf, fidx,
                       arp, aci, av, cf, cnum, fnum, prp, pci, pv, wrp, wci, wv, afc, hasf, err);
    return hipGetLastError();
}

hipError_t launch_interp_finish(hipStream_t st, int64_t n, const int8_t* cf, const int32_t* arp, const int32_t* aci,
                                const double* av, const double* wv, const int32_t* prp, const int32_t* pmap,
                                double* pv) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_interp_finish, dim3(static_cast<unsigned>((n + kRB - 1) / kRB)), dim3(kRB), 0, st, n, cf,
                       arp, aci, av, wv, prp, pmap, pv);
    return hipGetLastError();
}

hipError_t launch_fsai(hipStream_t st, int64_t n, const int32_t* arp, const int32_t* aci, const double* av,
                       const int32_t* grp, const int32_t* gci, double* gv, const int64_t* woff, double* work,
                       int* err) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fsai, dim3(static_cast<unsigned>((n + kRB - 1) / kRB)), dim3(kRB), 0, st, n, arp, aci, av,
                       grp, gci, gv, woff, work, err);
    return hipGetLastError();
}

hipError_t launch_spgemm_masked(hipStream_t st, int64_t nr, int64_t nnz, const int32_t* arp, const int32_t* aci,
                                const double* av, const int32_t* brp, const int32_t* bci, const double* bv,
                                const int32_t* crp, const int32_t* cci, double* cv) {
    if (nr <= 0 || nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spgemm_masked, dim3(grid_for(nnz)), dim3(kRB), 0, st, nr, nnz, arp, aci, av, brp, bci, bv,
                       crp, cci, cv);
    return hipGetLastError();
}

hipError_t launch_scale(hipStream_t st, int64_t n, double* v, double s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kRB), 0, st, n, v, s);
    return hipGetLastError();
}

hipError_t launch_split_strength(hipStream_t st, int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                                 const double* v, double theta, const int64_t* tmap, int8_t* smask, int8_t* tmask) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_strength, dim3(grid_for(n)), dim3(kRB), 0, st, n, rp, ci, v, theta, smask);
    hipLaunchKernelGGL(k_symmetric_mask, dim3(grid_for(nnz)), dim3(kRB), 0, st, nnz, tmap, smask, tmask);
    return hipGetLastError();
}

hipError_t launch_strong_dependants(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci,
                                   const int8_t* smask, int32_t* lam) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_strong_dependants, dim3(grid_for(n)), dim3(kRB), 0, st, n, rp, ci, smask, lam);
    return hipGetLastError();
}

hipError_t launch_mis_round(hipStream_t st, int64_t n, int d, const int32_t* rp, const int32_t* ci,
                            const int8_t* tmask, const int32_t* lam, const uint64_t* pri, int8_t* state, int* left) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mis_select, dim3(grid_for(n)), dim3(kRB), 0, st, n, d, rp, ci, tmask, lam, pri, state);
    hipLaunchKernelGGL(k_mis_remove, dim3(grid_for(n)), dim3(kRB), 0, st, n, d, rp, ci, tmask, state, left);
    return hipGetLastError();
}

hipError_t launch_split_diff(hipStream_t st, int64_t n, const int8_t* state, const int8_t* cf,
                             unsigned long long* count) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_diff, dim3(grid_for(n)), dim3(kRB), 0, st, n, state, cf, count);
    return hipGetLastError();
}

hipError_t launch_emin_project(hipStream_t st, int64_t n, const int32_t* rp, const int8_t* cf, const double* v,
                               double sign, double* out) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emin_project, dim3(grid_for(n)), dim3(kRB), 0, st, n, rp, cf, v, sign, out);
    return hipGetLastError();
}

hipError_t launch_emin_dinv(hipStream_t st, int64_t n, const int32_t* arp, const int32_t* aci, const double* av,
                            const int32_t* prp, double* dinv) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emin_dinv, dim3(grid_for(n)), dim3(kRB), 0, st, n, arp, aci, av, prp, dinv);
    return hipGetLastError();
}

hipError_t launch_emin_step(hipStream_t st, int64_t m, double alpha, const double* p, const double* q,
                            const double* dinv, double* w, double* r, double* z) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emin_step, dim3(grid_for(m)), dim3(kRB), 0, st, m, alpha, p, q, dinv, w, r, z);
    return hipGetLastError();
}

hipError_t launch_emin_dir(hipStream_t st, int64_t m, double beta, const double* z, double* p) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_emin_dir, dim3(grid_for(m)), dim3(kRB), 0, st, m, beta, z, p);
    return hipGetLastError();
}

hipError_t launch_mul(hipStream_t st, int64_t m, const double* a, const double* b, double* out) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mul, dim3(grid_for(m)), dim3(kRB), 0, st, m, a, b, out);
    return hipGetLastError();
}

hipError_t launch_sell_values(hipStream_t st, int64_t slots, int vs, const int64_t* pos, const double* v,
                              double* out64, float* out32) {
    if (slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sell_values, dim3(grid_for(slots * vs)), dim3(kRB), 0, st, slots, vs, pos, v, out64, out32);
    return hipGetLastError();
}

hipError_t launch_spmv(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* ci, const double* v,
                       const double* x, double* y, int64_t nnz) {
    if (n <= 0) return hipSuccess;
    if (nnz >= 32 * n) {   // long rows: a wavefront each
        hipLaunchKernelGGL(k_spmv_wave, dim3(static_cast<unsigned>((n + kRB / 64 - 1) / (kRB / 64))), dim3(kRB), 0,
                           st, n, rp, ci, v, x, y);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_spmv, dim3(static_cast<unsigned>((n + kRB - 1) / kRB)), dim3(kRB), 0, st, n, rp, ci, v, x,
                       y);
    return hipGetLastError();
}

hipError_t launch_power_dots(hipStream_t st, int64_t n, const double* v, const double* w, double* part, int nb,
                             double* out) {
    hipLaunchKernelGGL(k_dots2, dim3(nb), dim3(kRB), 0, st, n, v, w, part);
    hipLaunchKernelGGL(k_dots2_finish, dim3(1), dim3(64), 0, st, nb, part, out);
    return hipGetLastError();
}

hipError_t launch_normalise(hipStream_t st, int64_t n, const double* w, const double* dots, double* v) {
    hipLaunchKernelGGL(k_normalise, dim3(grid_for(n)), dim3(kRB), 0, st, n, w, dots, v);
    return hipGetLastError();
}

hipError_t launch_dense_inverse(hipStream_t st, int64_t n, int S, const int32_t* rp, const int32_t* ci,
                                const double* v, double* X, double* rowk, double* colk) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_densify, dim3(static_cast<unsigned>((n * S + kRB - 1) / kRB)), dim3(kRB), 0, st, n, S, rp,
                       ci, v, X);
    const unsigned gk = static_cast<unsigned>((n * S + kRB - 1) / kRB);
    const unsigned gu = static_cast<unsigned>((n * n * S + kRB - 1) / kRB);
    for (int64_t k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_gj_keep, dim3(gk), dim3(kRB), 0, st, n, S, k, X, rowk, colk);
        hipLaunchKernelGGL(k_gj_update, dim3(gu), dim3(kRB), 0, st, n, S, k, X, rowk, colk);
    }
    return hipGetLastError();
}

}  // namespace msp
