// Internal interface between the host API (mclbm_api.cpp) and the kernels
// (mclbm_kernels.hip).  Not part of the public C ABI.
#pragma once

#include "mclbm_device.hpp"

namespace mclbm {

// The state in row records (u_at): populations [ny][9][pitch] of double or
// float, or for 16-bit storage per lattice row four rows of 32-bit words (word
// w: population 2w in the low half, 2w + 1 in the high half) and one row of
// population 8 (16-bit values); u [ny][2][pitch] of double.
struct StepArgs {
    const void* fsrc;  // fc'_n
    void* fdst;        // fc'_{n+1}
    const double* usrc;  // u_n, [ny][2][pitch]
    double* udst;        // u_{n+1}
    Geometry g;
    Coef k;
    Walls w;
};

// What the per-node helpers need: the displacement field and the constants of
// the stress and source evaluation.
struct InitLike {
    const double* u;   // [ny][2][pitch]
    Geometry g;
    double inv_dx, inv_c2, sig_b[2], lam, mu, rho0;
    int bo;            // one-sided differences at the outermost nodes: 1 or 2
};

struct InitArgs {
    InitLike b;
    void* f;           // fc'_0 out
    const double* j0;  // [ny][2][pitch]
    double rho0, inv_c;
    double fscale;     // stored = population * fscale
};

struct ReadArgs {
    InitLike b;
    const void* f;     // fc'_n
    double* dst;       // [comp - c0][ny][nx] FP64
    int field;
    int c0, c1;        // components written: c0 <= comp < c1
    double c, s_from_sig;
    double finv;       // population = stored * finv
    double* partial;   // diagnostics: 8 doubles per block
    const double* sig; // sigma of the collision at t_n when it is held (the
                       // printed order's level n - 1), [2][ny][pitch]; else null
};

// The multi-pass step (second-order boundary differences, or the printed order
// of the time levels): the stress pass writes T, the source pass sigma, and the
// step kernel pulls, applies the walls, updates u and collides.
struct PassArgs {
    StepArgs s;
    double* T;              // stress pass output: T_n [4][ny][pitch]
    double* sig;            // source pass output: sigma_n [2][ny][pitch]
    const double* Tw;       // stresses the walls of step n use (T_n, or T_{n-1})
    const double* sig_c;    // sigma of the collision at t_n (sigma_n, or sigma_{n-1})
};

// The wall segments of a lattice: the nodes on its non-periodic sides (rows 0
// and ny - 1 whole, columns 0 and nx - 1 between them) in runs of kWallSeg along
// each side, one block per run (the wall rules of Sect. 3.3 in FP64; the march
// stores nothing there).
constexpr int kWallSeg = 64;
struct WallSegs {
    int nrow, ncol;  // segments per row side, per column side
    int total;
};
__host__ __device__ __forceinline__ WallSegs wall_segs(const Geometry& g) {
    WallSegs w;
    w.nrow = g.py ? 0 : (g.nx + kWallSeg - 1) / kWallSeg;
    const int h = g.py ? g.ny : g.ny - 2;
    w.ncol = g.px ? 0 : (h + kWallSeg - 1) / kWallSeg;
    w.total = 2 * w.nrow + 2 * w.ncol;
    return w;
}

// One simulation's share of one step of a batch: its step arguments, its work
// items [item0, item0 + nstrip * nchunk), its wall segments [seg0, seg0 +
// wall_segs(a.g).total) and whether it sits the step out (it has finished its
// steps in this round).
struct BatchEntry {
    StepArgs a;
    int nstrip, nchunk, chunk;
    int item0;
    int skip;
    int seg0;
};

// One step of a batch for one material: the simulations in item order.
struct BatchStep {
    int nsims, nitems, nsegs;
    int pad_;
    BatchEntry e[1];  // nsims entries (the table is allocated for the batch's maximum)
};
inline size_t batch_step_bytes(int max_sims) {
    return (sizeof(BatchStep) + (size_t)(max_sims - 1) * sizeof(BatchEntry) + 255) / 256 * 256;
}

// One lattice's displacement for the failure scan: u at [ny][2][pitch]; the
// scan raises flags[slot] if any u of a node is not finite or, when limit2 > 0,
// if |u|^2 exceeds limit2.
struct ScanEntry {
    const double* u;
    double limit2;
    int nx, ny, pitch, slot;
};
// scan n entries (a table in device memory) into flags (device memory, cleared
// by the caller); a fixed grid, so the launch costs the same for any batch
hipError_t launch_nanscan(const ScanEntry* tab, int n, uint32_t* flags, hipStream_t st);

// work items of one lattice's step in a batch: 64-column strips times row chunks
void march_shape(const Geometry& g, int* nstrip, int* nchunk, int* chunk);
// the step for every simulation of one material in the table at step (device
// memory, read by the kernels): the march on march_blocks blocks of four
// waves, one work item per wave, then the wall segments on wall_blocks
// blocks, one segment each; the grids must cover the table's items / 4 and
// segments (extra blocks end at once).  Graph-capturable: a captured launch
// serves any table that fits its grids.
hipError_t launch_batch_step(int prec, int material, const BatchStep* step, int march_blocks, int wall_blocks,
                             hipStream_t st);
// a grid of at least `need` blocks: a power of two, at least kMinBatchBlocks
// (so that a captured launch is re-captured only when a batch outgrows it by a
// factor of two)
constexpr int kMinBatchBlocks = 256;
inline int batch_grid(long long need) {
    long long b = kMinBatchBlocks;
    while (b < need) b *= 2;
    return (int)b;
}

}  // namespace mclbm

struct mclbm_sim;

namespace mclbm {

// host side, for the batching server: the batch entry of step n + k of s, the
// step counter advanced by k steps taken in batches, the thread's error message
void batch_entry(const mclbm_sim* s, int64_t k, BatchEntry* e);
void advance(mclbm_sim* s, int64_t k);
// the scan entry of s's displacement after k more steps
void scan_entry(const mclbm_sim* s, int64_t k, int slot, ScanEntry* e);
int set_error(int code, const char* msg);
// validation of a side program (the checks of mclbm_set_side)
int check_side_program(const void* spec);

// prec: PREC_F64 / F32 / F16 / BF16.  The step: one launch of march_kernel
// over every node off the non-periodic sides, carrying, when step_fused says
// so (every lattice with a non-periodic side), the wall blocks that update the
// nodes on them with the wall rules in FP64.
hipError_t launch_step(int prec, int material, const StepArgs& a, bool fused, hipStream_t st);
bool step_fused(int prec, const Geometry& g);
// the multi-pass step: stresses, source, step (three launches)
hipError_t launch_stress_pass(int material, const InitLike& b, double* T, hipStream_t st);
hipError_t launch_source_pass(const InitLike& b, const double* T, double* sig, hipStream_t st);
hipError_t launch_pass_step(int prec, const PassArgs& a, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t n4, hipStream_t st);
hipError_t launch_init(int prec, const InitArgs& a, hipStream_t st);
hipError_t launch_read(int prec, int material, const ReadArgs& a, hipStream_t st);
// diagnostics into out[0..4]; with watch non-null, also record step as the
// first bad step in *watch when the values are not finite and *watch < 0
hipError_t launch_diag(int prec, int material, const ReadArgs& a, double* out, int64_t* watch, int64_t step,
                       hipStream_t st);
int diag_blocks(const Geometry& g);
// the same diagnostics with the block partials and the result in the library's
// fixed device array (no workspace); copies the five totals to host_out and
// synchronises the stream
hipError_t launch_diag_noalloc(int prec, int material, ReadArgs a, double host_out[5], hipStream_t st);

}  // namespace mclbm
