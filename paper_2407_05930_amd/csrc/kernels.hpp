// Host-callable launchers of the HIP kernels (kernels.hip).  C is the padded
// column count of the multivectors (a power of two, 1..64).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace msp {

template <typename T>
hipError_t launch_spmm(hipStream_t st, int C, int64_t n, const int32_t* rp, const int32_t* ci, const T* va,
                       const T* X, T* Y, const T* Z, T alpha, T beta, const double* sigma, int S, int m);
template <typename T>
hipError_t launch_dot(hipStream_t st, int C, int64_t n, const T* X, const T* Y, double* partial, int nb,
                      double* out);

hipError_t launch_pcg_init(hipStream_t st, int C, const double* rr, const double* rz, const double* thr,
                           int* active, double* rho, int* iters, int* flags, double* rnorm);
hipError_t launch_pcg_alpha(hipStream_t st, int C, const double* pq, const int* active, const double* rho,
                            double* alpha, int* flags);
hipError_t launch_pcg_check(hipStream_t st, int C, const double* rr, const double* thr, int* active, int* iters,
                            int* flags, double* rnorm);
hipError_t launch_pcg_beta(hipStream_t st, int C, const double* rz, const double* rzold, const int* active,
                           double* rho, double* beta, int flexible);
hipError_t launch_pcg_update(hipStream_t st, int C, int64_t n, double* x, double* r, const double* p,
                             const double* q, const double* alpha);
hipError_t launch_pcg_pupdate(hipStream_t st, int C, int64_t n, double* p, const double* z, const double* beta,
                              const int* active);

hipError_t launch_qs_forward(hipStream_t st, int S, int64_t n_b, int m, int C, int64_t n, const int64_t* img,
                             const double* b, double* out);
hipError_t launch_qs_backward(hipStream_t st, int S, int64_t n_b, int m, int C, int64_t n, const int64_t* img,
                              const double* xh, double* x);
hipError_t launch_colnorm2(hipStream_t st, int64_t n, int m, const double* b, double* out);
hipError_t launch_thresholds(hipStream_t st, int C, int S, int m, double tol, const double* bn2, double* thr);

template <typename T>
hipError_t launch_dense(hipStream_t st, int C, int64_t nL, const double* Minv, const T* y, T* out);
template <typename T>
hipError_t launch_fill(hipStream_t st, int64_t len, T* p, T v);
template <typename TO, typename TI>
hipError_t launch_cast(hipStream_t st, int64_t len, const TI* a, TO* b);

}  // namespace msp
