// A stand-alone user of the mclbm C ABI, without Python or torch: it owns the
// device arena and the stream, as any caller does, runs a small lattice and
// writes the displacement to a file.
//
//   mclbm_demo OUT.bin [f64|f32] [nsteps]
//
// The lattice: 70 x 45 St. Venant-Kirchhoff, mu = 0.05, nu = 0.2, tau = 0.55;
// the left wall held, the right wall pulled by 0.5 dX over 200 steps and then
// held (Dirichlet), top and bottom traction-free (Neumann).  OUT.bin receives
// u as FP64 [2][ny][nx].  Exit status 0 on success; any ABI error is printed
// with mclbm_last_error() and ends the program with status 1.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <vector>

#include "mclbm.h"

static int check(int rc, const char* what) {
    if (rc != MCLBM_OK) {
        std::fprintf(stderr, "%s: status %d: %s\n", what, rc, mclbm_last_error());
        return 1;
    }
    return 0;
}

int main(int argc, char** argv) {
    if (argc < 2) {
        std::fprintf(stderr, "usage: %s OUT.bin [f64|f32] [nsteps]\n", argv[0]);
        return 2;
    }
    const bool f32 = argc > 2 && std::strcmp(argv[2], "f32") == 0;
    const long long nsteps = argc > 3 ? std::atoll(argv[3]) : 300;

    mclbm_params p;
    std::memset(&p, 0, sizeof p);
    p.nx = 70;
    p.ny = 45;
    p.material = MCLBM_SVK;
    p.precision = f32 ? MCLBM_F32 : MCLBM_F64;
    p.dx = 1.0;
    p.rho0 = 1.0;
    p.mu = 0.05;
    p.nu = 0.2;
    p.tau = 0.55;

    size_t bytes = 0;
    double dt = 0;
    if (check(mclbm_plan(&p, &bytes, nullptr, &dt), "mclbm_plan")) return 1;
    void* arena = nullptr;
    hipStream_t stream = nullptr;
    if (hipMalloc(&arena, bytes) != hipSuccess || hipStreamCreate(&stream) != hipSuccess) {
        std::fprintf(stderr, "device allocation or stream creation failed\n");
        return 1;
    }
    mclbm_sim* s = nullptr;
    int rc = check(mclbm_create(&p, arena, bytes, stream, &s), "mclbm_create");
    mclbm_side_spec held, pulled, free_;
    std::memset(&held, 0, sizeof held);
    held.bc = MCLBM_DIRICHLET;
    held.kind = MCLBM_LOAD_ZERO;
    pulled = held;
    pulled.kind = MCLBM_LOAD_DISP_RAMP;
    pulled.amp[0] = 0.5;
    pulled.t1 = 200;
    std::memset(&free_, 0, sizeof free_);
    free_.bc = MCLBM_NEUMANN;
    free_.kind = MCLBM_LOAD_ZERO;
    if (!rc) rc = check(mclbm_set_side(s, MCLBM_LEFT, &held), "mclbm_set_side");
    if (!rc) rc = check(mclbm_set_side(s, MCLBM_RIGHT, &pulled), "mclbm_set_side");
    if (!rc) rc = check(mclbm_set_side(s, MCLBM_BOTTOM, &free_), "mclbm_set_side");
    if (!rc) rc = check(mclbm_set_side(s, MCLBM_TOP, &free_), "mclbm_set_side");
    if (!rc) rc = check(mclbm_init(s, nullptr, nullptr, 0), "mclbm_init");
    if (!rc) rc = check(mclbm_step(s, nsteps), "mclbm_step");
    std::vector<double> u(2 * (size_t)p.nx * p.ny);
    if (!rc) rc = check(mclbm_read(s, MCLBM_FIELD_U, u.data(), 0), "mclbm_read");
    mclbm_diag_out d;
    if (!rc) rc = check(mclbm_diag(s, &d), "mclbm_diag");
    if (!rc) {
        FILE* f = std::fopen(argv[1], "wb");
        if (!f || std::fwrite(u.data(), sizeof(double), u.size(), f) != u.size()) {
            std::fprintf(stderr, "cannot write %s\n", argv[1]);
            rc = 1;
        }
        if (f) std::fclose(f);
        std::printf("{\"steps\": %lld, \"dt\": %.17g, \"max_u\": %.17g, \"momentum\": [%.17g, %.17g]}\n",
                    (long long)d.step, dt, d.max_u, d.momentum[0], d.momentum[1]);
    }
    if (s) mclbm_destroy(s);
    (void)hipStreamDestroy(stream);
    (void)hipFree(arena);
    return rc ? 1 : 0;
}
