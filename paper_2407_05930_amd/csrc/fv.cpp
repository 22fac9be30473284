// Finite-volume operator from base-mesh faces: assembly of the full matrix
// in the caller's ordering and the adjoint gradient with respect to kappa.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "refresh.hpp"

#define FVCHECK(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            throw msp::Error(e_ == hipErrorOutOfMemory ? MSP_ERR_OOM : MSP_ERR_HIP,               \
                             std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    } while (0)

struct msp_fv {
    int s = 0, S = 1;
    int64_t n = 0, n_b = 0, nf = 0;
    std::vector<int64_t> ca, cb, img;
    std::vector<int8_t> kind, axis;
    std::vector<double> area, da, db;
    // cell -> incident faces (CSR over base cells)
    std::vector<int64_t> cfp;
    std::vector<int32_t> cfi;
    int device = -1;
    std::vector<void*> dev;
    int64_t *d_cfp = nullptr, *d_img = nullptr, *d_ca = nullptr, *d_cb = nullptr;
    int32_t* d_cfi = nullptr;
    int8_t *d_kind = nullptr, *d_axis = nullptr;
    double *d_area = nullptr, *d_da = nullptr, *d_db = nullptr;
    // device assembly: per position of the assembled matrix, the face whose -T
    // it holds (>= 0) or the base cell whose diagonal it holds (-(i+1)); T per
    // face and the diagonal per base cell as work arrays
    int32_t* d_slot = nullptr;
    int64_t nnz = 0;
    double *d_T = nullptr, *d_diag = nullptr;
    ~msp_fv() {
        if (device >= 0) {
            (void)hipSetDevice(device);
            for (void* p : dev) (void)hipFree(p);
        }
    }
    template <typename T>
    T* up(const std::vector<T>& h) {
        void* p = nullptr;
        FVCHECK(hipMalloc(&p, sizeof(T) * std::max<size_t>(1, h.size())));
        dev.push_back(p);
        if (!h.empty()) FVCHECK(hipMemcpy(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
        return static_cast<T*>(p);
    }
};

static double face_T(const msp_fv* f, int64_t q, const double* kap) {
    const double ka = kap[f->ca[q]];
    switch (f->kind[q]) {
        case 0: return f->area[q] / (f->da[q] / ka + f->db[q] / kap[f->cb[q]]);
        case 1: return f->area[q] * ka / f->da[q];
        default: return f->area[q] * ka / (2.0 * f->da[q]);
    }
}

namespace msp {

void fv_create(const msp_faces* F, const msp_symmap* map, int device, msp_fv** out) {
    if (!F || !map || !out || !F->cell_a || !F->cell_b || !F->kind || !F->axis || !F->area || !F->dist_a ||
        !F->dist_b || !map->img)
        throw Error(MSP_ERR_ARG, "null face arrays or map");
    if (map->s < 0 || map->s > 6 || map->n_b <= 0) throw Error(MSP_ERR_ARG, "bad map");
    std::unique_ptr<msp_fv> f(new msp_fv());
    f->s = map->s;
    f->S = 1 << map->s;
    f->n_b = map->n_b;
    f->n = map->n_b << map->s;
    f->nf = F->nf;
    const int64_t nf = F->nf;
    f->ca.assign(F->cell_a, F->cell_a + nf);
    f->cb.assign(F->cell_b, F->cell_b + nf);
    f->kind.assign(F->kind, F->kind + nf);
    f->axis.assign(F->axis, F->axis + nf);
    f->area.assign(F->area, F->area + nf);
    f->da.assign(F->dist_a, F->dist_a + nf);
    f->db.assign(F->dist_b, F->dist_b + nf);
    f->img.assign(map->img, map->img + f->n_b * f->S);
    std::vector<char> seen(f->n, 0);
    for (int64_t v : f->img) {
        if (v < 0 || v >= f->n || seen[v]) throw Error(MSP_ERR_BAD_MAP, "symmetry map is not a permutation");
        seen[v] = 1;
    }
    for (int64_t q = 0; q < nf; ++q) {
        if (f->ca[q] < 0 || f->ca[q] >= f->n_b) throw Error(MSP_ERR_ARG, "face cell out of range");
        if (f->kind[q] == 0 && (f->cb[q] < 0 || f->cb[q] >= f->n_b)) throw Error(MSP_ERR_ARG, "interior face cell");
        if (f->kind[q] < 0 || f->kind[q] > 2) throw Error(MSP_ERR_ARG, "face kind");
        if (f->kind[q] == 2 && (f->axis[q] < 0 || f->axis[q] >= f->s)) throw Error(MSP_ERR_ARG, "mirror face axis");
        if (!(f->area[q] > 0.0) || !(f->da[q] > 0.0) || (f->kind[q] == 0 && !(f->db[q] > 0.0)))
            throw Error(MSP_ERR_ARG, "face area and distances must be positive");
    }
    // cell -> faces (each interior face is listed for both of its cells)
    f->cfp.assign(f->n_b + 1, 0);
    for (int64_t q = 0; q < nf; ++q) {
        f->cfp[f->ca[q] + 1]++;
        if (f->kind[q] == 0) f->cfp[f->cb[q] + 1]++;
    }
    for (int64_t i = 0; i < f->n_b; ++i) f->cfp[i + 1] += f->cfp[i];
    f->cfi.resize(f->cfp[f->n_b]);
    std::vector<int64_t> pos(f->cfp.begin(), f->cfp.end() - 1);
    for (int64_t q = 0; q < nf; ++q) {
        f->cfi[pos[f->ca[q]]++] = static_cast<int32_t>(q);
        if (f->kind[q] == 0) f->cfi[pos[f->cb[q]]++] = static_cast<int32_t>(q);
    }
    if (device >= 0) {
        FVCHECK(hipSetDevice(device));
        f->device = device;
        f->d_cfp = f->up(f->cfp);
        f->d_cfi = f->up(f->cfi);
        f->d_img = f->up(f->img);
        f->d_ca = f->up(f->ca);
        f->d_cb = f->up(f->cb);
        f->d_kind = f->up(f->kind);
        f->d_axis = f->up(f->axis);
        f->d_area = f->up(f->area);
        f->d_da = f->up(f->da);
        f->d_db = f->up(f->db);
    }
    *out = f.release();
}

int64_t fv_nnz(const msp_fv* f) {
    int64_t per = 0;   // entries per image: diagonal + interior couplings + mirror couplings
    per += f->n_b;
    for (int64_t q = 0; q < f->nf; ++q) {
        if (f->kind[q] == 0) per += 2;
        else if (f->kind[q] == 2) per += 1;
    }
    return per * f->S;
}

void fv_assemble(const msp_fv* f, const double* kap, int64_t* rp, int32_t* ci, double* va) {
    if (!kap || !rp || !ci || !va) throw Error(MSP_ERR_ARG, "null array");
    for (int64_t i = 0; i < f->n_b; ++i)
        if (!(kap[i] > 0.0)) throw Error(MSP_ERR_ARG, "kappa must be positive");
    const int S = f->S;
    std::vector<double> T(f->nf), diag(f->n_b, 0.0);
    for (int64_t q = 0; q < f->nf; ++q) T[q] = face_T(f, q, kap);
    for (int64_t i = 0; i < f->n_b; ++i)
        for (int64_t e = f->cfp[i]; e < f->cfp[i + 1]; ++e) diag[i] += T[f->cfi[e]];
    // rows in the caller's ordering: row img[i*S + a] of base cell i, image a
    std::vector<int64_t> cnt(f->n + 1, 0);
    for (int64_t i = 0; i < f->n_b; ++i) {
        const int64_t deg = 1 + (f->cfp[i + 1] - f->cfp[i]);
        int64_t walls = 0;
        for (int64_t e = f->cfp[i]; e < f->cfp[i + 1]; ++e) walls += f->kind[f->cfi[e]] == 1;
        for (int a = 0; a < S; ++a) cnt[f->img[i * S + a] + 1] = deg - walls;
    }
    for (int64_t g = 0; g < f->n; ++g) cnt[g + 1] += cnt[g];
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = 0; i < f->n_b; ++i)
        for (int a = 0; a < S; ++a) {
            const int64_t g = f->img[i * S + a];
            row.clear();
            row.emplace_back(static_cast<int32_t>(g), diag[i]);
            for (int64_t e = f->cfp[i]; e < f->cfp[i + 1]; ++e) {
                const int64_t q = f->cfi[e];
                if (f->kind[q] == 0) {
                    const int64_t o = f->ca[q] == i ? f->cb[q] : f->ca[q];
                    row.emplace_back(static_cast<int32_t>(f->img[o * S + a]), -T[q]);
                } else if (f->kind[q] == 2) {
                    row.emplace_back(static_cast<int32_t>(f->img[i * S + (a ^ (1 << f->axis[q]))]), -T[q]);
                }
            }
            std::sort(row.begin(), row.end(),
                      [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                          return x.first < y.first;
                      });
            int64_t p = cnt[g];
            for (auto& pr : row) {
                ci[p] = pr.first;
                va[p] = pr.second;
                ++p;
            }
        }
    std::copy(cnt.begin(), cnt.end(), rp);
}

// The positions of the host assembly, built once: each row of image a of base
// cell i holds the diagonal and one entry per interior or mirror face of i,
// sorted by column.
static void fv_build_slots(msp_fv* f) {
    if (f->nf >= (int64_t(1) << 31) || f->n_b >= (int64_t(1) << 31))
        throw Error(MSP_ERR_UNSUPPORTED, "device assembly needs fewer than 2^31 faces and base cells");
    const int S = f->S;
    std::vector<int64_t> cnt(f->n + 1, 0);
    for (int64_t i = 0; i < f->n_b; ++i) {
        int64_t deg = 1;
        for (int64_t e = f->cfp[i]; e < f->cfp[i + 1]; ++e) deg += f->kind[f->cfi[e]] != 1;
        for (int a = 0; a < S; ++a) cnt[f->img[i * S + a] + 1] = deg;
    }
    for (int64_t g = 0; g < f->n; ++g) cnt[g + 1] += cnt[g];
    std::vector<int32_t> slot(cnt[f->n]);
    std::vector<std::pair<int32_t, int32_t>> row;
    for (int64_t i = 0; i < f->n_b; ++i)
        for (int a = 0; a < S; ++a) {
            const int64_t g = f->img[i * S + a];
            row.clear();
            row.emplace_back(static_cast<int32_t>(g), static_cast<int32_t>(-(i + 1)));
            for (int64_t e = f->cfp[i]; e < f->cfp[i + 1]; ++e) {
                const int64_t q = f->cfi[e];
                if (f->kind[q] == 0) {
                    const int64_t o = f->ca[q] == i ? f->cb[q] : f->ca[q];
                    row.emplace_back(static_cast<int32_t>(f->img[o * S + a]), static_cast<int32_t>(q));
                } else if (f->kind[q] == 2) {
                    row.emplace_back(static_cast<int32_t>(f->img[i * S + (a ^ (1 << f->axis[q]))]),
                                     static_cast<int32_t>(q));
                }
            }
            std::sort(row.begin(), row.end(),
                      [](const std::pair<int32_t, int32_t>& x, const std::pair<int32_t, int32_t>& y) {
                          return x.first < y.first;
                      });
            int64_t p = cnt[g];
            for (auto& pr : row) slot[p++] = pr.second;
        }
    f->nnz = cnt[f->n];
    f->d_slot = f->up(slot);
    f->d_T = f->up(std::vector<double>(std::max<int64_t>(1, f->nf)));
    f->d_diag = f->up(std::vector<double>(f->n_b));
}

void fv_assemble_device(msp_fv* f, const double* d_kap, double* d_val, hipStream_t st) {
    if (f->device < 0) throw Error(MSP_ERR_ARG, "operator was created without a device");
    if (!d_kap || !d_val) throw Error(MSP_ERR_ARG, "null array");
    FVCHECK(hipSetDevice(f->device));
    if (!f->d_slot) fv_build_slots(f);
    FVCHECK(launch_fv_values(st, f->nf, f->n_b, f->nnz, f->d_ca, f->d_cb, f->d_kind, f->d_area, f->d_da, f->d_db,
                             f->d_cfp, f->d_cfi, f->d_slot, d_kap, f->d_T, f->d_diag, d_val));
}

void fv_free(msp_fv* f) { delete f; }

void fv_kappa_grad(msp_fv* f, const double* d_kap, int m, const double* d_lam, const double* d_p, double* d_grad,
                   hipStream_t st) {
    if (f->device < 0) throw Error(MSP_ERR_ARG, "operator was created without a device");
    if (m <= 0 || !d_kap || !d_lam || !d_p || !d_grad) throw Error(MSP_ERR_ARG, "bad gradient arguments");
    FVCHECK(hipSetDevice(f->device));
    FVCHECK(launch_kappa_grad(st, f->n_b, f->S, f->n, m, f->d_cfp, f->d_cfi, f->d_img, f->d_ca, f->d_cb, f->d_kind,
                              f->d_axis, f->d_area, f->d_da, f->d_db, d_kap, d_lam, d_p, d_grad));
}

}  // namespace msp
