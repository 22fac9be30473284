// Default options (plain C++: the host setup's sanitizer build links it
// without the HIP runtime).
#include <cstring>

#include "msp.h"

extern "C" int msp_default_opts(msp_opts* o) {
    if (!o) return MSP_ERR_ARG;
    std::memset(o, 0, sizeof(*o));
    o->precision = MSP_FP64;
    o->pc = MSP_PC_AMGR;
    o->lrc_k = 0;
    o->dist = 2;
    o->theta = 0.25;
    o->jacobi0 = 3;
    o->trunc0 = 0.05;
    o->jacobi = 1;
    o->coarse_max = 2560;
    o->max_levels = 20;
    o->max_ratio = 0.8;
    o->tol = 1e-10;
    o->maxit = 1000;
    o->device = 0;
    o->seed = 240705930ull;
    o->coarse64 = 0;
    o->nu1 = 1;
    o->nu2 = 1;
    o->amgs_light = 0;
    o->schur_tau = 0.01;
    o->true_residual = 0;
    o->afsai_nnz = 0;
    o->emin_steps = 0;
    return MSP_OK;
}
