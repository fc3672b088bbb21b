// Host side of the mclbm C ABI: parameter validation, the arena layout, the wall
// load programs and the launch sequence of the step.  No device allocation: the
// caller provides the arena and the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mclbm.h"
#include "mclbm_internal.hpp"

#define MCLBM_EXPORT extern "C" __attribute__((visibility("default")))

using namespace mclbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(MCLBM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int pitch;
    bool multipass;  // second-order boundary differences or the printed order
    bool listing;    // the printed order: S and T of the previous level are state
    size_t f_bytes, u_bytes, part_bytes, out_bytes, watch_bytes, t_bytes, s_bytes;
    size_t off_f[2], off_u[2], off_part, off_out, off_watch, off_t[2], off_s[2], total;
};

// bytes per node of one population buffer: nine FP64 or FP32 values, or nine
// 16-bit values (per lattice row four rows of two per 32-bit word and one row of 16-bit values)
size_t pop_bytes_per_node(int precision) {
    return precision == MCLBM_F64 ? 72 : (precision == MCLBM_F32 ? 36 : 18);
}

Layout layout_of(const mclbm_params& p) {
    Layout L;
    L.pitch = (p.nx + 63) / 64 * 64;
    const size_t plane = (size_t)p.ny * L.pitch;
    L.f_bytes = align_up(pop_bytes_per_node(p.precision) * plane);
    L.u_bytes = align_up(2 * plane * 8);
    Geometry g{p.nx, p.ny, L.pitch, 0, 0, (long long)plane};
    L.part_bytes = align_up((size_t)diag_blocks(g) * 8 * sizeof(double));
    L.out_bytes = align_up(8 * sizeof(double));
    L.watch_bytes = align_up(8 * sizeof(int64_t));
    L.listing = p.time_levels == 1;
    L.multipass = L.listing || p.boundary_order == 2;
    // the multi-pass step holds T (4 components) and sigma (2) in FP64; the
    // printed order keeps the previous level's beside the current one
    L.t_bytes = L.multipass ? align_up(4 * plane * 8) : 0;
    L.s_bytes = L.multipass ? align_up(2 * plane * 8) : 0;
    size_t o = 0;
    L.off_f[0] = o; o += L.f_bytes;
    L.off_f[1] = o; o += L.f_bytes;
    L.off_u[0] = o; o += L.u_bytes;
    L.off_u[1] = o; o += L.u_bytes;
    L.off_part = o; o += L.part_bytes;
    L.off_out = o; o += L.out_bytes;
    L.off_watch = o; o += L.watch_bytes;
    for (int k = 0; k < 2; k++) {
        L.off_t[k] = o; o += (k == 0 || L.listing) ? L.t_bytes : 0;
        L.off_s[k] = o; o += (k == 0 || L.listing) ? L.s_bytes : 0;
    }
    if (!L.listing) { L.off_t[1] = L.off_t[0]; L.off_s[1] = L.off_s[0]; }
    L.total = o;
    return L;
}

int check_params(const mclbm_params* p) {
    if (!p) return fail(MCLBM_EINVAL, "params is NULL");
    if (p->nx < 3 || p->ny < 3) return fail(MCLBM_EINVAL, "nx and ny must be >= 3 (got %d x %d)", p->nx, p->ny);
    if (p->precision < MCLBM_F64 || p->precision > MCLBM_BF16)
        return fail(MCLBM_EINVAL, "unknown precision %d", p->precision);
    // the device addresses a displacement buffer (two FP64 values per node of the
    // pitched lattice) through one 32-bit buffer range
    {
        const int64_t plane = (int64_t)p->ny * ((p->nx + 63) / 64 * 64);
        if (plane * 2 * 8 >= ((int64_t)1 << 32))
            return fail(MCLBM_EINVAL, "lattice of %d x %d nodes too large for one device buffer range "
                        "(a displacement buffer must stay below 4 GiB)", p->nx, p->ny);
        // and one lattice row's record of populations (nine FP64 rows at most)
        // through another
        const int64_t pitch = (p->nx + 63) / 64 * 64;
        if (pitch * 9 * 8 >= ((int64_t)1 << 32))
            return fail(MCLBM_EINVAL, "lattice rows of %d nodes too long for one device buffer range "
                        "(a row of populations must stay below 4 GiB)", p->nx);
    }
    if (!(p->dx > 0) || !(p->rho0 > 0) || !(p->mu > 0))
        return fail(MCLBM_EINVAL, "dx, rho0 and mu must be positive");
    if (!(p->tau > 0.5)) return fail(MCLBM_EINVAL, "tau must exceed 0.5 (got %g)", p->tau);
    if (!(p->tau_plus == 0.0 || p->tau_plus > 0.5))
        return fail(MCLBM_EINVAL, "tau_plus must be 0 (BGK) or exceed 0.5 (got %g)", p->tau_plus);
    if (!(p->growth_limit >= 0.0 && std::isfinite(p->growth_limit)))
        return fail(MCLBM_EINVAL, "growth_limit must be finite and >= 0 (got %g)", p->growth_limit);
    if (!(p->nu > -1.0 && p->nu < 0.5)) return fail(MCLBM_EINVAL, "nu must lie in (-1, 0.5) (got %g)", p->nu);
    if (p->material < MCLBM_SVK || p->material > MCLBM_LINEAR)
        return fail(MCLBM_EINVAL, "unknown material %d", p->material);
    if (!std::isfinite(p->body[0]) || !std::isfinite(p->body[1]))
        return fail(MCLBM_EINVAL, "body force must be finite");
    if (p->extrap != 0 && p->extrap != 1) return fail(MCLBM_EINVAL, "extrap must be 0 or 1 (got %d)", p->extrap);
    if (p->corner < 0 || p->corner > 2) return fail(MCLBM_EINVAL, "corner must be 0, 1 or 2 (got %d)", p->corner);
    if (p->boundary_order < 0 || p->boundary_order > 2)
        return fail(MCLBM_EINVAL, "boundary_order must be 1 or 2 (0 means 1; got %d)", p->boundary_order);
    if (p->time_levels != 0 && p->time_levels != 1)
        return fail(MCLBM_EINVAL, "time_levels must be 0 or 1 (got %d)", p->time_levels);
    if (p->diag_every < 0) return fail(MCLBM_EINVAL, "diag_every must be >= 0 (got %d)", p->diag_every);
    if (p->reserved_ != 0) return fail(MCLBM_EINVAL, "reserved_ must be 0");
    return MCLBM_OK;
}

// lattice speed c = sqrt(3) c_s, c_s = sqrt(mu/rho0) (Sect. 3.2); dt = dX / c
double lattice_speed(const mclbm_params& p) { return std::sqrt(3.0 * p.mu / p.rho0); }

constexpr int64_t kMaxTable = (int64_t)1 << 26;

int check_side(const mclbm_side_spec* s) {
    if (!s) return fail(MCLBM_EINVAL, "side spec is NULL");
    if (s->bc < MCLBM_DIRICHLET || s->bc > MCLBM_PERIODIC) return fail(MCLBM_EINVAL, "unknown wall type %d", s->bc);
    if (s->kind < MCLBM_LOAD_ZERO || s->kind > MCLBM_LOAD_TABLE)
        return fail(MCLBM_EINVAL, "unknown load program %d", s->kind);
    if (s->kind == MCLBM_LOAD_TABLE) {
        if (!s->table || s->table_len < 1 || s->table_len > kMaxTable)
            return fail(MCLBM_EINVAL, "a TABLE program needs a table of 1..%lld entries", (long long)kMaxTable);
        for (int64_t i = 0; i < s->table_len; i++)
            if (!std::isfinite(s->table[i])) return fail(MCLBM_EINVAL, "TABLE entry %lld is not finite", (long long)i);
    }
    if (s->kind == MCLBM_LOAD_DISP_RAMP && s->bc != MCLBM_DIRICHLET)
        return fail(MCLBM_EINVAL, "DISP_RAMP prescribes a wall speed and needs a Dirichlet side");
    const bool need_t1 = s->kind == MCLBM_LOAD_DISP_RAMP || s->kind == MCLBM_LOAD_LINEAR_RAMP ||
                         s->kind == MCLBM_LOAD_SIN2_RAMP || s->kind == MCLBM_LOAD_SIN_PULSE;
    if (need_t1 && !(s->t1 > 0)) return fail(MCLBM_EINVAL, "load program %d needs t1 > 0", s->kind);
    if ((s->kind == MCLBM_LOAD_GAUSS || s->kind == MCLBM_LOAD_RICKER) && !(s->width > 0))
        return fail(MCLBM_EINVAL, "load program %d needs width > 0", s->kind);
    if (!std::isfinite(s->amp[0]) || !std::isfinite(s->amp[1])) return fail(MCLBM_EINVAL, "load amplitude must be finite");
    return MCLBM_OK;
}

}  // namespace

struct mclbm_sim {
    mclbm_params p;
    Layout L;
    char* arena;
    hipStream_t stream;
    Geometry g;
    Coef k;
    double dt;
    mclbm_side_spec side[4];
    std::vector<double> table[4];  // TABLE programs (side[i].table points here)
    int cur;       // which of the two population / displacement buffers is current
    int sp;        // the printed order: which T / sigma buffer holds level n - 1
    int64_t n;     // steps since init
    bool inited;
};

namespace {

// Time program of a wall load at step n.
double load_scale(const mclbm_side_spec& s, double n) {
    switch (s.kind) {
    case MCLBM_LOAD_TABLE: {
        const int64_t k = (int64_t)n;
        return s.table[k < s.table_len ? k : s.table_len - 1];
    }
    case MCLBM_LOAD_ZERO: return 0.0;
    case MCLBM_LOAD_CONST: return 1.0;
    case MCLBM_LOAD_LINEAR_RAMP: return n < s.t1 ? n / s.t1 : 1.0;
    case MCLBM_LOAD_SIN2_RAMP: {
        if (n >= s.t1) return 1.0;
        const double v = std::sin(M_PI * n / (2.0 * s.t1));
        return v * v;
    }
    case MCLBM_LOAD_SIN_PULSE: return n < s.t1 ? std::sin(M_PI * n / s.t1) : 0.0;
    case MCLBM_LOAD_GAUSS: {
        if (n > s.t1) return 0.0;
        const double d = n - s.t0;
        return std::exp(-d * d / (2.0 * s.width * s.width));
    }
    case MCLBM_LOAD_RICKER: {
        if (n >= s.t1) return 0.0;
        const double d2 = (n - s.t0) * (n - s.t0);
        return 2.0 / std::sqrt(3.0 * s.width * std::sqrt(M_PI)) * (1.0 - d2 / s.width) *
               std::exp(-0.5 * d2 / s.width);
    }
    default: return 0.0;
    }
}

Walls walls_at(const mclbm_sim* s, int64_t n) {
    Walls w;
    for (int i = 0; i < 4; i++) {
        const mclbm_side_spec& sp = s->side[i];
        w.bc[i] = sp.bc;
        double k;
        if (sp.kind == MCLBM_LOAD_DISP_RAMP)  // j* = rho0 * wall speed while the ramp runs
            k = (double)n < sp.t1 ? s->p.rho0 / (sp.t1 * s->dt) : 0.0;
        else
            k = load_scale(sp, (double)n);
        w.val[i][0] = sp.amp[0] * k;
        w.val[i][1] = sp.amp[1] * k;
    }
    return w;
}

int check_pairs(const mclbm_sim* s) {
    const bool l = s->side[MCLBM_LEFT].bc == MCLBM_PERIODIC, r = s->side[MCLBM_RIGHT].bc == MCLBM_PERIODIC;
    const bool b = s->side[MCLBM_BOTTOM].bc == MCLBM_PERIODIC, t = s->side[MCLBM_TOP].bc == MCLBM_PERIODIC;
    if (l != r) return fail(MCLBM_EINVAL, "periodic left/right sides must be set as a pair");
    if (b != t) return fail(MCLBM_EINVAL, "periodic bottom/top sides must be set as a pair");
    return MCLBM_OK;
}

void* at(const mclbm_sim* s, size_t off) { return s->arena + off; }

InitLike base_args(const mclbm_sim* s, const double* u) {
    InitLike b;
    b.u = u;
    b.g = s->g;
    b.inv_dx = s->k.inv_dx;
    b.inv_c2 = s->k.inv_c2;
    b.sig_b[0] = s->k.sig_b[0];
    b.sig_b[1] = s->k.sig_b[1];
    b.lam = s->k.lam;
    b.mu = s->k.mu;
    b.rho0 = s->k.rho0;
    b.bo = s->p.boundary_order == 2 ? 2 : 1;
    return b;
}

// copy a compact [2][ny][nx] FP64 field into a buffer of row records, [ny][2][pitch]
int put_field2(mclbm_sim* s, double* dst, const double* src, int on_device) {
    const size_t plane = (size_t)s->g.plane;
    if (!src) {
        HIP_TRY(hipMemsetAsync(dst, 0, 2 * plane * sizeof(double), s->stream));
        return MCLBM_OK;
    }
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(hipMemsetAsync(dst, 0, 2 * plane * sizeof(double), s->stream));
    for (int c = 0; c < 2; c++)
        HIP_TRY(hipMemcpy2DAsync(dst + (size_t)c * s->g.pitch, 2 * (size_t)s->g.pitch * sizeof(double),
                                 src + (size_t)c * s->g.nx * s->g.ny, (size_t)s->g.nx * sizeof(double),
                                 (size_t)s->g.nx * sizeof(double), (size_t)s->g.ny, kind, s->stream));
    return MCLBM_OK;
}

// the first-bad-step record of the diagnostics watch: -1, written by a small
// host copy (ordered on the stream before any step)
int reset_watch(mclbm_sim* s) {
    static const int64_t none[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    HIP_TRY(hipMemcpyAsync(at(s, s->L.off_watch), none, sizeof none, hipMemcpyHostToDevice, s->stream));
    return MCLBM_OK;
}

}  // namespace

MCLBM_EXPORT int mclbm_plan(const mclbm_params* p, size_t* arena_bytes, size_t* align, double* dt_out) {
    const int rc = check_params(p);
    if (rc) return rc;
    const Layout L = layout_of(*p);
    if (arena_bytes) *arena_bytes = L.total;
    if (align) *align = kAlign;
    if (dt_out) *dt_out = p->dx / lattice_speed(*p);
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_create(const mclbm_params* p, void* arena, size_t arena_bytes, void* stream,
                              mclbm_sim** out) {
    const int rc = check_params(p);
    if (rc) return rc;
    if (!out) return fail(MCLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!arena) return fail(MCLBM_EINVAL, "arena is NULL");
    if ((uintptr_t)arena % kAlign) return fail(MCLBM_ETOOSMALL, "arena must be %zu-byte aligned", kAlign);
    const Layout L = layout_of(*p);
    if (arena_bytes < L.total)
        return fail(MCLBM_ETOOSMALL, "arena has %zu bytes, %zu needed", arena_bytes, L.total);
    mclbm_sim* s = new (std::nothrow) mclbm_sim();
    if (!s) return fail(MCLBM_EINVAL, "out of host memory");
    s->p = *p;
    s->L = L;
    s->arena = static_cast<char*>(arena);
    s->stream = static_cast<hipStream_t>(stream);
    s->g = Geometry{p->nx, p->ny, L.pitch, 0, 0, (long long)p->ny * L.pitch};
    const double c = lattice_speed(*p);
    s->dt = p->dx / c;
    s->k.omega = 1.0 / p->tau;
    s->k.omega_p = p->tau_plus > 0.5 ? 1.0 / p->tau_plus : s->k.omega;
    s->k.c = c;
    s->k.inv_c = 1.0 / c;
    s->k.inv_c2 = 1.0 / (c * c);
    s->k.inv_dx = 1.0 / p->dx;
    s->k.ucoef = p->dx / (2.0 * p->rho0);
    s->k.sig_b[0] = p->rho0 * p->body[0] * p->dx * s->k.inv_c2;
    s->k.sig_b[1] = p->rho0 * p->body[1] * p->dx * s->k.inv_c2;
    s->k.s_from_sig = c * c / p->dx;
    s->k.lam = 2.0 * p->mu * p->nu / (1.0 - 2.0 * p->nu);  // plane strain
    s->k.mu = p->mu;
    s->k.rho0 = p->rho0;
    // FP16 storage keeps the populations times 2^(12 - floor(log2 rho0)): |f| up to
    // about 16 rho0 stays below the FP16 maximum, and down to about 1.5e-8 rho0 in
    // its normal range
    s->k.fscale = p->precision == MCLBM_F16 ? std::ldexp(1.0, 12 - std::ilogb(p->rho0)) : 1.0;
    s->k.finv = 1.0 / s->k.fscale;
    s->k.extrap = p->extrap;
    s->k.corner = p->corner;
    for (int i = 0; i < 4; i++) {
        std::memset(&s->side[i], 0, sizeof(mclbm_side_spec));
        s->side[i].bc = MCLBM_NEUMANN;
        s->side[i].kind = MCLBM_LOAD_ZERO;
    }
    s->cur = 0;
    s->sp = 0;
    s->n = 0;
    s->inited = false;
    *out = s;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_set_side(mclbm_sim* s, int side, const mclbm_side_spec* spec) {
    if (!s) return fail(MCLBM_EINVAL, "handle is NULL");
    if (side < MCLBM_LEFT || side > MCLBM_TOP) return fail(MCLBM_EINVAL, "unknown side %d", side);
    const int rc = check_side(spec);
    if (rc) return rc;
    if (s->inited && (spec->bc == MCLBM_PERIODIC) != (s->side[side].bc == MCLBM_PERIODIC))
        return fail(MCLBM_ESTATE, "periodicity of a side can only change before mclbm_init");
    s->side[side] = *spec;
    if (spec->kind == MCLBM_LOAD_TABLE) {
        s->table[side].assign(spec->table, spec->table + spec->table_len);
        s->side[side].table = s->table[side].data();
    } else {
        s->table[side].clear();
        s->side[side].table = nullptr;
        s->side[side].table_len = 0;
    }
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_init(mclbm_sim* s, const double* u0, const double* j0, int on_device) {
    if (!s) return fail(MCLBM_EINVAL, "handle is NULL");
    int rc = check_pairs(s);
    if (rc) return rc;
    s->g.px = s->side[MCLBM_LEFT].bc == MCLBM_PERIODIC;
    s->g.py = s->side[MCLBM_BOTTOM].bc == MCLBM_PERIODIC;
    s->cur = 0;
    double* u = static_cast<double*>(at(s, s->L.off_u[0]));
    double* stage = static_cast<double*>(at(s, s->L.off_u[1]));
    if ((rc = put_field2(s, u, u0, on_device))) return rc;
    if ((rc = put_field2(s, stage, j0, on_device))) return rc;
    InitArgs a;
    a.b = base_args(s, u);
    a.f = at(s, s->L.off_f[0]);
    a.j0 = stage;
    a.rho0 = s->p.rho0;
    a.inv_c = s->k.inv_c;
    a.fscale = s->k.fscale;
    HIP_TRY(launch_init(s->p.precision, a, s->stream));
    s->sp = 0;
    if (s->L.listing) {
        // the printed order enters its first step with S and T of u0 as level -1
        double* T = static_cast<double*>(at(s, s->L.off_t[0]));
        double* sg = static_cast<double*>(at(s, s->L.off_s[0]));
        HIP_TRY(launch_stress_pass(s->p.material, a.b, T, s->stream));
        HIP_TRY(launch_source_pass(a.b, T, sg, s->stream));
    }
    if ((rc = reset_watch(s))) return rc;
    s->n = 0;
    s->inited = true;
    return MCLBM_OK;
}

namespace {

StepArgs step_args(const mclbm_sim* s) {
    StepArgs a;
    a.fsrc = at(s, s->L.off_f[s->cur]);
    a.fdst = at(s, s->L.off_f[1 - s->cur]);
    a.usrc = static_cast<const double*>(at(s, s->L.off_u[s->cur]));
    a.udst = static_cast<double*>(at(s, s->L.off_u[1 - s->cur]));
    a.g = s->g;
    a.k = s->k;
    a.w = walls_at(s, s->n);
    return a;
}

int check_steppable(const mclbm_sim* s, int64_t nsteps) {
    if (!s) return fail(MCLBM_EINVAL, "handle is NULL");
    if (!s->inited) return fail(MCLBM_ESTATE, "step before mclbm_init");
    if (nsteps < 0) return fail(MCLBM_EINVAL, "nsteps must be >= 0");
    return MCLBM_OK;
}

// arguments of the per-node read-out and diagnostics kernels at t_n
ReadArgs read_args(const mclbm_sim* s) {
    ReadArgs a;
    a.b = base_args(s, static_cast<const double*>(at(s, s->L.off_u[s->cur])));
    a.f = at(s, s->L.off_f[s->cur]);
    a.dst = nullptr;
    a.field = 0;
    a.c0 = 0;
    a.c1 = 4;
    a.c = s->k.c;
    a.s_from_sig = s->k.s_from_sig;
    a.finv = s->k.finv;
    a.partial = static_cast<double*>(at(s, s->L.off_part));
    // the printed order's collision at t_n uses the held sigma of level n - 1
    a.sig = s->L.listing ? static_cast<const double*>(at(s, s->L.off_s[s->sp])) : nullptr;
    return a;
}

// one step on the stream: march_kernel carrying the wall blocks (the event,
// when set, is recorded after it), or the three passes of the multi-pass step.
// (The wall blocks as a kernel of their own on a second stream beside the march
// made the 8192^2 step 2 % slower in FP32 and halved the step rate of small
// lattices, whose steps last tens of microseconds.)
hipError_t launch_one_step(mclbm_sim* s, hipEvent_t between = nullptr) {
    const StepArgs a = step_args(s);
    if (!s->L.multipass) {
        const bool fused = step_fused(s->p.precision, s->g);
        hipError_t e = launch_step(s->p.precision, s->p.material, a, fused, s->stream);
        if (e == hipSuccess && between) e = hipEventRecord(between, s->stream);
        return e;
    }
    PassArgs pa;
    pa.s = a;
    // level n goes to the buffers not holding level n - 1
    const int wn = s->L.listing ? 1 - s->sp : 0;
    pa.T = static_cast<double*>(at(s, s->L.off_t[wn]));
    pa.sig = static_cast<double*>(at(s, s->L.off_s[wn]));
    pa.Tw = static_cast<const double*>(at(s, s->L.off_t[s->L.listing ? s->sp : wn]));
    pa.sig_c = static_cast<const double*>(at(s, s->L.off_s[s->L.listing ? s->sp : wn]));
    const InitLike b = base_args(s, a.usrc);
    hipError_t e = launch_stress_pass(s->p.material, b, pa.T, s->stream);
    if (e == hipSuccess) e = launch_source_pass(b, pa.T, pa.sig, s->stream);
    if (e == hipSuccess) e = launch_pass_step(s->p.precision, pa, s->stream);
    if (e == hipSuccess && between) e = hipEventRecord(between, s->stream);
    return e;
}

void advance_one(mclbm_sim* s) {
    s->cur = 1 - s->cur;
    if (s->L.listing) s->sp = 1 - s->sp;
    s->n++;
}

}  // namespace

MCLBM_EXPORT int mclbm_step(mclbm_sim* s, int64_t nsteps) {
    if (int e = check_steppable(s, nsteps)) return e;
    for (int64_t i = 0; i < nsteps; i++) {
        HIP_TRY(launch_one_step(s));
        advance_one(s);
        if (s->p.diag_every > 0 && s->n % s->p.diag_every == 0) {
            // the watch: diagnostics on the device, the first non-finite step kept
            const ReadArgs a = read_args(s);
            HIP_TRY(launch_diag(s->p.precision, s->p.material, a, static_cast<double*>(at(s, s->L.off_out)),
                                static_cast<int64_t*>(at(s, s->L.off_watch)), s->n, s->stream));
        }
    }
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_step_checked(mclbm_sim* s, int64_t nsteps, int64_t every, int64_t* steps_run) {
    if (steps_run) *steps_run = 0;
    if (int e = check_steppable(s, nsteps)) return e;
    if (every < 1) return fail(MCLBM_EINVAL, "every must be >= 1");
    // the scan's table entry and its flag sit in the arena's diagnostics result area
    // (the watch of diag_every writes there too, earlier on the same stream)
    char* area = static_cast<char*>(at(s, s->L.off_out));
    static_assert(sizeof(ScanEntry) + sizeof(uint32_t) <= 8 * sizeof(double), "result area too small");
    int64_t done = 0;
    while (done < nsteps) {
        const int64_t k = std::min<int64_t>(every, nsteps - done);
        if (int rc = mclbm_step(s, k)) return rc;
        done += k;
        struct {
            ScanEntry e;
            uint32_t flag;
        } h;
        std::memset(&h, 0, sizeof h);
        scan_entry(s, 0, 0, &h.e);
        uint32_t flag = 0;
        HIP_TRY(hipMemcpyAsync(area, &h, sizeof h, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(launch_nanscan(reinterpret_cast<const ScanEntry*>(area), 1,
                               reinterpret_cast<uint32_t*>(area + offsetof(decltype(h), flag)), s->stream));
        HIP_TRY(hipMemcpyAsync(&flag, area + offsetof(decltype(h), flag), sizeof flag, hipMemcpyDeviceToHost,
                               s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (steps_run) *steps_run = done;
        if (flag)
            return fail(MCLBM_EUNSTABLE, "displacement not finite%s by step %lld",
                        s->p.growth_limit > 0.0 ? " or above the growth limit" : "", (long long)s->n);
    }
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_step_timed(mclbm_sim* s, int64_t nsteps, double* ms_step, double* ms_main) {
    if (int e = check_steppable(s, nsteps)) return e;
    if (nsteps < 1 || nsteps > 100000) return fail(MCLBM_EINVAL, "nsteps must be in 1..100000");
    if (!ms_step && !ms_main) return fail(MCLBM_EINVAL, "both output pointers are NULL");
    // a[i] before step i's launches, b[i] after its main kernel, a[nsteps] after the last step
    std::vector<hipEvent_t> a((size_t)(nsteps + 1), nullptr), b((size_t)nsteps, nullptr);
    int rc = MCLBM_OK;
    for (auto* v : {&a, &b})
        for (auto& e : *v)
            if (rc == MCLBM_OK && hipEventCreate(&e) != hipSuccess) {
                e = nullptr;
                rc = fail(MCLBM_EHIP, "hipEventCreate failed");
            }
    for (int64_t i = 0; rc == MCLBM_OK && i < nsteps; i++) {
        hipError_t e = hipEventRecord(a[i], s->stream);
        if (e == hipSuccess) e = launch_one_step(s, b[i]);
        if (e != hipSuccess) {
            rc = fail(MCLBM_EHIP, "step launch failed: %s", hipGetErrorString(e));
            break;
        }
        advance_one(s);
    }
    if (rc == MCLBM_OK && hipEventRecord(a[nsteps], s->stream) != hipSuccess)
        rc = fail(MCLBM_EHIP, "hipEventRecord failed");
    if (rc == MCLBM_OK && hipStreamSynchronize(s->stream) != hipSuccess)
        rc = fail(MCLBM_EHIP, "hipStreamSynchronize failed");
    double tstep = 0, tmain = 0;
    for (int64_t k = 0; rc == MCLBM_OK && k < nsteps; k++) {
        float m1 = 0, m2 = 0;
        if (hipEventElapsedTime(&m1, a[k], a[k + 1]) != hipSuccess ||
            hipEventElapsedTime(&m2, a[k], b[k]) != hipSuccess)
            rc = fail(MCLBM_EHIP, "hipEventElapsedTime failed");
        tstep += m1;
        tmain += m2;
    }
    for (auto* v : {&a, &b})
        for (auto e : *v)
            if (e) (void)hipEventDestroy(e);
    if (rc != MCLBM_OK) return rc;
    if (ms_step) *ms_step = tstep / nsteps;
    if (ms_main) *ms_main = tmain / nsteps;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_copy(void* dst, const void* src, size_t nbytes, void* stream) {
    if (nbytes % 4) return fail(MCLBM_EINVAL, "nbytes must be a multiple of 4");
    if (nbytes && (!dst || !src)) return fail(MCLBM_EINVAL, "NULL buffer");
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 4)
        return fail(MCLBM_EINVAL, "buffers must be 4-byte aligned");
    HIP_TRY(launch_copy(dst, src, nbytes / 4, static_cast<hipStream_t>(stream)));
    return MCLBM_OK;
}

// ---- internals for the batching server (mclbm_serve.cpp) -------------------------------------

namespace mclbm {

// the arguments of step n + k of s (the populations and displacement ping-pong
// by step parity) and its work items
void batch_entry(const mclbm_sim* s, int64_t k, BatchEntry* e) {
    const int c = (s->cur + (int)(k & 1)) & 1;
    e->a.fsrc = at(s, s->L.off_f[c]);
    e->a.fdst = at(s, s->L.off_f[1 - c]);
    e->a.usrc = static_cast<const double*>(at(s, s->L.off_u[c]));
    e->a.udst = static_cast<double*>(at(s, s->L.off_u[1 - c]));
    e->a.g = s->g;
    e->a.k = s->k;
    e->a.w = walls_at(s, s->n + k);
    march_shape(s->g, &e->nstrip, &e->nchunk, &e->chunk);
    e->skip = 0;
    e->seg0 = 0;
}

void scan_entry(const mclbm_sim* s, int64_t k, int slot, ScanEntry* e) {
    const int c = (s->cur + (int)(k & 1)) & 1;
    e->u = static_cast<const double*>(at(s, s->L.off_u[c]));
    e->limit2 = s->p.growth_limit * s->p.growth_limit;
    e->nx = s->g.nx;
    e->ny = s->g.ny;
    e->pitch = s->g.pitch;
    e->slot = slot;
}

// record k steps taken outside mclbm_step
void advance(mclbm_sim* s, int64_t k) {
    s->n += k;
    s->cur = (s->cur + (int)(k & 1)) & 1;
}

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

int check_side_program(const void* spec) { return check_side(static_cast<const mclbm_side_spec*>(spec)); }

}  // namespace mclbm

MCLBM_EXPORT int64_t mclbm_stepno(const mclbm_sim* s) { return s ? s->n : -1; }

MCLBM_EXPORT int mclbm_field_components(int field) {
    switch (field) {
    case MCLBM_FIELD_U: case MCLBM_FIELD_J: case MCLBM_FIELD_S: return 2;
    case MCLBM_FIELD_R: return 1;
    case MCLBM_FIELD_PI: return 3;
    case MCLBM_FIELD_H: case MCLBM_FIELD_P: return 4;
    default: return 0;
    }
}

MCLBM_EXPORT int mclbm_read(mclbm_sim* s, int field, double* dst, int on_device) {
    if (!s) return fail(MCLBM_EINVAL, "handle is NULL");
    if (!s->inited) return fail(MCLBM_ESTATE, "mclbm_read before mclbm_init");
    const int nc = mclbm_field_components(field);
    if (!nc) return fail(MCLBM_EINVAL, "unknown field %d", field);
    if (!dst) return fail(MCLBM_EINVAL, "dst is NULL");
    ReadArgs a = read_args(s);
    a.field = field;
    a.partial = nullptr;
    const size_t plane_out = (size_t)s->g.nx * s->g.ny;
    if (on_device) {
        a.dst = dst;
        a.c0 = 0;
        a.c1 = nc;
        HIP_TRY(launch_read(s->p.precision, s->p.material, a, s->stream));
    } else {
        // a host destination is staged in the idle population buffer, as many
        // components per pass as it holds (at least two: it has 18 B or more per
        // node of the pitched lattice); each pass's copy is ordered before the
        // next pass overwrites the staging
        double* stage = static_cast<double*>(at(s, s->L.off_f[1 - s->cur]));
        const int per = (int)std::min<size_t>((size_t)nc, s->L.f_bytes / (plane_out * sizeof(double)));
        if (per < 1) return fail(MCLBM_EINVAL, "staging buffer too small");
        for (int c0 = 0; c0 < nc; c0 += per) {
            a.dst = stage;
            a.c0 = c0;
            a.c1 = std::min(nc, c0 + per);
            HIP_TRY(launch_read(s->p.precision, s->p.material, a, s->stream));
            HIP_TRY(hipMemcpyAsync(dst + (size_t)c0 * plane_out, stage, (size_t)(a.c1 - c0) * plane_out * sizeof(double),
                                   hipMemcpyDeviceToHost, s->stream));
        }
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return MCLBM_OK;
}

namespace {

// mclbm_diag_out from the five totals and the watch record; the status
int diag_result(mclbm_sim* s, const double h[5], int64_t first_bad, mclbm_diag_out* out) {
    std::memset(out, 0, sizeof *out);
    out->step = s->n;
    out->first_bad_step = s->p.diag_every > 0 ? first_bad : -1;
    out->momentum[0] = h[0];
    out->momentum[1] = h[1];
    out->ekin = h[2];
    out->max_u = std::sqrt(h[3]);
    out->nonfinite = h[4] != 0.0;
    out->growth = s->p.growth_limit > 0.0 && out->max_u > s->p.growth_limit;
    // c_d^2 = (lambda + 2 mu) / rho0 against c^2 = 3 mu / rho0 (first-order
    // boundary differences: c_d <= c, nu <= 1/4) or 4 c^2 (second order:
    // c_d <= 2 c, nu <= 5/11)
    const double lam = 2.0 * s->p.mu * s->p.nu / (1.0 - 2.0 * s->p.nu);
    out->cfl_excess = s->p.boundary_order == 2 ? lam + 2.0 * s->p.mu > 12.0 * s->p.mu : lam > s->p.mu;
    if (out->nonfinite) return fail(MCLBM_EUNSTABLE, "non-finite u or j at step %lld", (long long)s->n);
    if (out->growth)
        return fail(MCLBM_EUNSTABLE, "max |u| %g above the growth limit %g at step %lld", out->max_u,
                    s->p.growth_limit, (long long)s->n);
    return MCLBM_OK;
}

}  // namespace

MCLBM_EXPORT int mclbm_diag(mclbm_sim* s, mclbm_diag_out* out) {
    if (!s) return fail(MCLBM_EINVAL, "handle is NULL");
    if (!out) return fail(MCLBM_EINVAL, "out is NULL");
    if (!s->inited) return fail(MCLBM_ESTATE, "mclbm_diag before mclbm_init");
    const ReadArgs a = read_args(s);
    double* dout = static_cast<double*>(at(s, s->L.off_out));
    HIP_TRY(launch_diag(s->p.precision, s->p.material, a, dout, nullptr, 0, s->stream));
    double h[5];
    int64_t first_bad = -1;
    HIP_TRY(hipMemcpyAsync(h, dout, sizeof h, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(&first_bad, at(s, s->L.off_watch), sizeof first_bad, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return diag_result(s, h, first_bad, out);
}

MCLBM_EXPORT int mclbm_diag_noalloc(mclbm_sim* s, mclbm_diag_out* out) {
    if (!s) return fail(MCLBM_EINVAL, "handle is NULL");
    if (!out) return fail(MCLBM_EINVAL, "out is NULL");
    if (!s->inited) return fail(MCLBM_ESTATE, "mclbm_diag_noalloc before mclbm_init");
    ReadArgs a = read_args(s);
    a.partial = nullptr;  // the partials go to the library's fixed array
    double h[5];
    HIP_TRY(launch_diag_noalloc(s->p.precision, s->p.material, a, h, s->stream));
    int64_t first_bad = -1;
    HIP_TRY(hipMemcpyAsync(&first_bad, at(s, s->L.off_watch), sizeof first_bad, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return diag_result(s, h, first_bad, out);
}

namespace {

// checkpoint header: 64 bytes ahead of the state
struct CkptHeader {
    char magic[8];      // "MCLBMCK1"
    int32_t version;    // 2: the state in row records
    int32_t nx, ny, precision, material, time_levels;
    int64_t step;
    uint64_t f_bytes, u_bytes, extra_bytes;  // populations, displacement, held level n - 1
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header layout");
constexpr char kMagic[8] = {'M', 'C', 'L', 'B', 'M', 'C', 'K', '1'};
constexpr int32_t kVersion = 2;

size_t extra_bytes(const mclbm_sim* s) { return s->L.listing ? s->L.t_bytes + s->L.s_bytes : 0; }

CkptHeader header_of(const mclbm_sim* s) {
    CkptHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, kMagic, sizeof kMagic);
    h.version = kVersion;
    h.nx = s->p.nx;
    h.ny = s->p.ny;
    h.precision = s->p.precision;
    h.material = s->p.material;
    h.time_levels = s->p.time_levels;
    h.step = s->n;
    h.f_bytes = s->L.f_bytes;
    h.u_bytes = s->L.u_bytes;
    h.extra_bytes = extra_bytes(s);
    return h;
}

}  // namespace

MCLBM_EXPORT size_t mclbm_state_bytes(const mclbm_sim* s) {
    return s ? sizeof(CkptHeader) + s->L.f_bytes + s->L.u_bytes + extra_bytes(s) : 0;
}

MCLBM_EXPORT int mclbm_save(mclbm_sim* s, void* dst, size_t dst_bytes, int on_device) {
    if (!s || !dst) return fail(MCLBM_EINVAL, "NULL argument");
    if (!s->inited) return fail(MCLBM_ESTATE, "mclbm_save before mclbm_init");
    if (dst_bytes < mclbm_state_bytes(s))
        return fail(MCLBM_EINVAL, "checkpoint buffer has %zu bytes, %zu needed", dst_bytes, mclbm_state_bytes(s));
    char* d = static_cast<char*>(dst);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const CkptHeader h = header_of(s);
    size_t o = sizeof h;
    HIP_TRY(hipMemcpyAsync(d + o, at(s, s->L.off_f[s->cur]), s->L.f_bytes, kind, s->stream));
    o += s->L.f_bytes;
    HIP_TRY(hipMemcpyAsync(d + o, at(s, s->L.off_u[s->cur]), s->L.u_bytes, kind, s->stream));
    o += s->L.u_bytes;
    if (s->L.listing) {
        HIP_TRY(hipMemcpyAsync(d + o, at(s, s->L.off_t[s->sp]), s->L.t_bytes, kind, s->stream));
        o += s->L.t_bytes;
        HIP_TRY(hipMemcpyAsync(d + o, at(s, s->L.off_s[s->sp]), s->L.s_bytes, kind, s->stream));
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (on_device) HIP_TRY(hipMemcpy(d, &h, sizeof h, hipMemcpyHostToDevice));
    else std::memcpy(d, &h, sizeof h);
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_load(mclbm_sim* s, const void* src, size_t src_bytes, int on_device) {
    if (!s || !src) return fail(MCLBM_EINVAL, "NULL argument");
    if (src_bytes < sizeof(CkptHeader)) return fail(MCLBM_EINVAL, "checkpoint of %zu bytes has no header", src_bytes);
    int rc = check_pairs(s);
    if (rc) return rc;
    const char* d = static_cast<const char*>(src);
    CkptHeader h;
    if (on_device) HIP_TRY(hipMemcpy(&h, d, sizeof h, hipMemcpyDeviceToHost));
    else std::memcpy(&h, d, sizeof h);
    const CkptHeader want = header_of(s);
    if (std::memcmp(h.magic, kMagic, sizeof kMagic) != 0 || h.version != kVersion)
        return fail(MCLBM_EINVAL, "not an mclbm checkpoint (magic or version)");
    if (h.nx != want.nx || h.ny != want.ny || h.precision != want.precision || h.material != want.material ||
        h.time_levels != want.time_levels || h.f_bytes != want.f_bytes || h.u_bytes != want.u_bytes ||
        h.extra_bytes != want.extra_bytes)
        return fail(MCLBM_EINVAL,
                    "checkpoint of a %d x %d lattice (precision %d, material %d, time levels %d) does not match "
                    "this simulation (%d x %d, %d, %d, %d)", h.nx, h.ny, h.precision, h.material, h.time_levels,
                    want.nx, want.ny, want.precision, want.material, want.time_levels);
    if (h.step < 0) return fail(MCLBM_EINVAL, "checkpoint step counter is negative");
    if (src_bytes < mclbm_state_bytes(s))
        return fail(MCLBM_EINVAL, "checkpoint has %zu bytes, %zu needed", src_bytes, mclbm_state_bytes(s));
    s->g.px = s->side[MCLBM_LEFT].bc == MCLBM_PERIODIC;
    s->g.py = s->side[MCLBM_BOTTOM].bc == MCLBM_PERIODIC;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    s->cur = 0;
    s->sp = 0;
    size_t o = sizeof h;
    HIP_TRY(hipMemcpyAsync(at(s, s->L.off_f[0]), d + o, s->L.f_bytes, kind, s->stream));
    o += s->L.f_bytes;
    HIP_TRY(hipMemcpyAsync(at(s, s->L.off_u[0]), d + o, s->L.u_bytes, kind, s->stream));
    o += s->L.u_bytes;
    if (s->L.listing) {
        HIP_TRY(hipMemcpyAsync(at(s, s->L.off_t[0]), d + o, s->L.t_bytes, kind, s->stream));
        o += s->L.t_bytes;
        HIP_TRY(hipMemcpyAsync(at(s, s->L.off_s[0]), d + o, s->L.s_bytes, kind, s->stream));
    }
    if ((rc = reset_watch(s))) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->n = h.step;
    s->inited = true;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_destroy(mclbm_sim* s) {
    delete s;
    return MCLBM_OK;
}

MCLBM_EXPORT const char* mclbm_last_error(void) { return g_err.c_str(); }
