// Internal interface between the host API (mclbm_api.cpp) and the kernels
// (mclbm_kernels.hip).  Not part of the public C ABI.
#pragma once

#include "mclbm_device.hpp"

namespace mclbm {

// Populations: [9][ny + 1][pitch] of double or float, or for 16-bit storage four
// planes of 32-bit words (word w: population 2w in the low half, 2w + 1 in the
// high half) followed by one plane of population 8 (16-bit values).
struct StepArgs {
    const void* fsrc;  // fc'_n
    void* fdst;        // fc'_{n+1}
    const double* usrc;  // u_n, [2][ny][pitch]
    double* udst;        // u_{n+1}
    Geometry g;
    Coef k;
    Walls w;
};

// What the per-node helpers need: the displacement field and the constants of
// the stress and source evaluation.
struct InitLike {
    const double* u;   // [2][ny][pitch]
    Geometry g;
    double inv_dx, inv_c2, sig_b[2], lam, mu, rho0;
};

struct InitArgs {
    InitLike b;
    void* f;           // fc'_0 out
    const double* j0;  // [2][ny][pitch]
    double rho0, inv_c;
    double fscale;     // stored = population * fscale
};

struct ReadArgs {
    InitLike b;
    const void* f;     // fc'_n
    double* dst;       // [comp][ny][nx] FP64
    int field;
    double c, s_from_sig;
    double finv;       // population = stored * finv
    double* partial;   // diagnostics: 8 doubles per block
};

// prec: PREC_F64 / F32 / F16 / BF16.  One launch: march_kernel over every node,
// walls included.
hipError_t launch_step(int prec, int material, const StepArgs& a, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t n4, hipStream_t st);
hipError_t launch_init(int prec, const InitArgs& a, hipStream_t st);
hipError_t launch_read(int prec, int material, const ReadArgs& a, hipStream_t st);
hipError_t launch_diag(int prec, int material, const ReadArgs& a, double* out, hipStream_t st);
int diag_blocks(const Geometry& g);

}  // namespace mclbm
