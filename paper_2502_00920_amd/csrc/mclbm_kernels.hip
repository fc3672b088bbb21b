// HIP kernels of the moment-chain LBM step for gfx950 (MI355X).
//
// One time step of Algorithm 1 (with the stresses taken at the current level,
// Sect. 3.1).  The state between steps is
//   fc' = the post-collision populations WITHOUT the forcing term, and u (FP64).
// This works because the forcing enters the BGK collision additively:
//   f - (f - f_eq(r, j, Pi))/tau* + (1 - 1/(2 tau*)) psi(S) dt
//     = (1 - 1/tau*) f + f_eq(r, sum c f, Pi)/tau* + dt psi(S)
// (j = sum c f + dt/2 S enters f_eq linearly), so the step n can add
// dt psi(S_n) while it pulls the populations, once S_n is known from u_n:
//   1. T_n = P(H) + Pi(H) from finite differences of u_n
//   2. sigma_n = dt S_n / c = (dt/c)(rho0 b + Div T_n)
//   3. pull f(t_{n+1})_q = fc'_q(X - e_q) + dt psi_q(S_n(X - e_q)); at walls the
//      modified bounce-back / anti-bounce-back rules of Sect. 3.3 from the
//      node's own post-collision populations and T_n(X)
//   4. u_{n+1} = u_n + dt/(2 rho0) (j(t_{n+1}) + j(t_n)), both j carrying S_n
//   5. fc'_{n+1} = (1 - omega) f + omega f_eq(r, M1, M2)
// A step is two launches: march_kernel updates every node as an interior node
// (one pass over HBM), then wall_kernel recomputes the nodes on non-periodic
// walls (0.05 % of an 8192^2 lattice) with the wall rules.
// HBM traffic per node and step: 9 populations read and written, u read and
// written (FP64): 176 B in FP64, 104 B in FP32 storage.
#include "mclbm_internal.hpp"

namespace mclbm {

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of
// work items, so that the halo rows and columns neighbours re-read sit in the
// same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
    const int q = nblk / 8, r = nblk % 8;
    const int xcd = bid % 8, k = bid / 8;
    return xcd * q + min(xcd, r) + k;
}

// wrap an index that is at most one period out of range
__device__ __forceinline__ int wrap1(int g, int n) { return g < 0 ? g + n : (g >= n ? g - n : g); }

// Raw buffer access: a wave-uniform resource (base, size in bytes), a
// wave-uniform SGPR offset and a 32-bit byte offset per lane.  Three component
// planes share one resource, so that a step needs eight resources in all.
constexpr uint32_t kRsrcWord3 = 0x00020000;  // gfx9-family buffer format word
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, (int)kRsrcWord3);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t ob, uint32_t so, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, ob, so, 0));
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t ob, uint32_t so, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, ob, so, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t ob, uint32_t so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, ob, so, 0);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t ob, uint32_t so, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, ob, so, 0);
}

// ---- step: interior nodes, y-marching ------------------------------------------------------
//
// Each wave owns a strip of MO = 58 columns (lanes 3..60, halo lanes 0..2 and
// 61..63) and marches down a chunk of rows.  At iteration r it holds in
// registers the rows r..r+3 of u, r..r+2 of T, r-1..r+1 of sigma and r-1..r+1
// of the populations; x neighbours come from lane shuffles, y neighbours from
// the rows it holds.  No LDS, no barriers, no branches on wall nodes (whose
// results wall_kernel overwrites).  Every population and u value of the strip
// is loaded once (the next rows one iteration ahead), plus the halo columns and
// the rows that prime the pipeline of a chunk.

constexpr int MH = 3, MO = 64 - 2 * MH;

template <typename V>
__device__ __forceinline__ V from_prev(V v) { return __shfl_up(v, 1); }    // value of lane l-1
template <typename V>
__device__ __forceinline__ V from_next(V v) { return __shfl_down(v, 1); }  // value of lane l+1

template <typename T, int MAT>
__global__ __launch_bounds__(256) void march_kernel(StepArgs a, int nstrip, int nchunk, int chunk) {
    const Geometry g = a.g;
    const int lane = threadIdx.x & 63;
    // the work item is uniform across the wave: keep it (and all row arithmetic) scalar
    const int item = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6));
    if (item >= nstrip * nchunk) return;
    const int strip = item % nstrip, chk = item / nstrip;
    const int gxu = strip * MO - MH + lane;  // unwrapped column of this lane
    // The loop below is straight-line: every lane issues every load and store.
    // Loads outside the lattice read a clamped address; their values only reach
    // links into wall nodes, which wall_kernel recomputes, and the one-sided
    // differences at the lattice edge never read them.  Stores of halo lanes and
    // of the rows that prime the pipeline go to row ny of each plane, which
    // nothing reads.  With no skipped memory operation the loads of the next rows
    // stay in flight across an iteration and the stores are never waited for.
    const bool xin = g.px ? true : (gxu >= 0 && gxu < g.nx);
    const int x = g.px ? wrap(gxu, g.nx) : min(max(gxu, 0), g.nx - 1);
    // population loads of lanes 0, 1, 62, 63 are never used: give them the
    // address of lane 2 / 61, which the memory pipeline merges
    const int lp = min(max(lane, MH - 1), MH + MO);
    const int gxp = strip * MO - MH + lp;
    const int xp = g.px ? wrap(gxp, g.nx) : min(max(gxp, 0), g.nx - 1);
    const bool own = lane >= MH && lane < MH + MO && gxu < g.nx;
    const bool atL = xin && at_low(x, g.px), atR = xin && at_high(x, g.nx, g.px);
    const int yc = chk * chunk, ye = min(yc + chunk, g.ny);
    const size_t plane = (size_t)g.plane;
    const uint32_t pbT = (uint32_t)(plane * sizeof(T)), pbD = (uint32_t)(plane * sizeof(double));
    const T* fs = reinterpret_cast<const T*>(a.fsrc);
    T* fd = reinterpret_cast<T*>(a.fdst);
    // resources: populations q in [3k, 3k + 3) at SGPR offset (q - 3k) planes
    const __amdgpu_buffer_rsrc_t rs0 = rsrc(fs, 3 * pbT), rs1 = rsrc(fs + 3 * plane, 3 * pbT),
                                 rs2 = rsrc(fs + 6 * plane, 3 * pbT);
    const __amdgpu_buffer_rsrc_t rd0 = rsrc(fd, 3 * pbT), rd1 = rsrc(fd + 3 * plane, 3 * pbT),
                                 rd2 = rsrc(fd + 6 * plane, 3 * pbT);
    const __amdgpu_buffer_rsrc_t rus = rsrc(a.usrc, 2 * pbD), rud = rsrc(a.udst, 2 * pbD);
    const double idx = a.k.inv_dx;
    const T ic2 = T(a.k.inv_c2), sbx = T(a.k.sig_b[0]), sby = T(a.k.sig_b[1]);
    const T lam = T(a.k.lam), mu = T(a.k.mu);
    const uint32_t trash = (uint32_t)(g.ny * g.pitch + lane);  // row ny: written, never read

    // row r (uniform) -> row to address, and whether it lies in the lattice
    auto rowc = [&](int r, bool& ok) -> int {
        if (g.py) { ok = true; return wrap(r, g.ny); }
        ok = r >= 0 && r < g.ny;
        return min(max(r, 0), g.ny - 1);
    };
    auto load_u = [&](int r, double v[2]) {
        bool ok;
        const int rr = rowc(r, ok);
        const uint32_t ob = (uint32_t)(rr * g.pitch + x) * (uint32_t)sizeof(double);
        v[0] = bload(rus, ob, 0u, 0.0);
        v[1] = bload(rus, ob, pbD, 0.0);
    };
    auto load_f = [&](int r, T f[9]) {
        bool ok;
        const int rr = rowc(r, ok);
        const uint32_t ob = (uint32_t)(rr * g.pitch + xp) * (uint32_t)sizeof(T);
#pragma unroll
        for (int q = 0; q < 9; q++)
            f[q] = bload(q < 3 ? rs0 : (q < 6 ? rs1 : rs2), ob, (uint32_t)(q % 3) * pbT, T(0));
    };
    // the stores of one node: u (2 x FP64) and the nine populations
    auto store_node = [&](uint32_t node, double vx, double vy, const T fn[9]) {
        const uint32_t ou = node * (uint32_t)sizeof(double), of = node * (uint32_t)sizeof(T);
        bstore(rud, ou, 0u, vx);
        bstore(rud, ou, pbD, vy);
#pragma unroll
        for (int q = 0; q < 9; q++)
            bstore(q < 3 ? rd0 : (q < 6 ? rd1 : rd2), of, (uint32_t)(q % 3) * pbT, fn[q]);
    };
    // T = P(H) + Pi(H) at row r from u at rows r-1, r, r+1 of this lane
    auto stress = [&](int r, const double um[2], const double u0[2], const double up[2], T t[4]) {
        const double lx = from_prev(u0[0]), rx = from_next(u0[0]);
        const double ly = from_prev(u0[1]), ry = from_next(u0[1]);
        bool ok;
        const int rr = rowc(r, ok);
        const double ax = atL ? u0[0] : lx, bx = atR ? u0[0] : rx;
        const double ay = atL ? u0[1] : ly, by = atR ? u0[1] : ry;
        const double fx = (atL || atR) ? idx : 0.5 * idx;
        const bool lo = !g.py && rr == 0, hi = !g.py && rr == g.ny - 1;
        const double cx = lo ? u0[0] : um[0], dx = hi ? u0[0] : up[0];
        const double cy = lo ? u0[1] : um[1], dy = hi ? u0[1] : up[1];
        const double fy = (lo || hi) ? idx : 0.5 * idx;
        T e[4];
        excess_stress<T, MAT>(T((bx - ax) * fx), T((dx - cx) * fy), T((by - ay) * fx), T((dy - cy) * fy),
                              lam, mu, e);
        const bool v = ok && xin;
#pragma unroll
        for (int c = 0; c < 4; c++) t[c] = v ? e[c] : T(0);
    };
    // sigma = dt S / c at row r from T at rows r-1, r, r+1 of this lane
    auto sigma = [&](int r, const T tm[4], const T t0[4], const T tp[4], T sg[2]) {
        const T lxx = from_prev(t0[0]), rxx = from_next(t0[0]);
        const T lyx = from_prev(t0[2]), ryx = from_next(t0[2]);
        bool ok;
        const int rr = rowc(r, ok);
        const T axx = atL ? t0[0] : lxx, bxx = atR ? t0[0] : rxx;
        const T ayx = atL ? t0[2] : lyx, byx = atR ? t0[2] : ryx;
        const T fx = (atL || atR) ? T(1) : T(0.5);
        const bool lo = !g.py && rr == 0, hi = !g.py && rr == g.ny - 1;
        const T cxy = lo ? t0[1] : tm[1], dxy = hi ? t0[1] : tp[1];
        const T cyy = lo ? t0[3] : tm[3], dyy = hi ? t0[3] : tp[3];
        const T fy = (lo || hi) ? T(1) : T(0.5);
        const bool v = ok && xin;
        const T s0 = ic2 * ((bxx - axx) * fx + (dxy - cxy) * fy) + sbx;
        const T s1 = ic2 * ((byx - ayx) * fx + (dyy - cyy) * fy) + sby;
        sg[0] = v ? s0 : T(0);
        sg[1] = v ? s1 : T(0);
    };

    // Pipeline state at iteration r: u rows r..r+2 (U0..U2), T rows r, r+1,
    // sigma rows r-1, r, populations rows r-1, r.  Two prefetch sets (A, B)
    // alternate: the rows an iteration consumes were loaded two iterations
    // earlier, so each wave keeps two rows of loads in flight.
    double U0[2], U1[2], U2[2], tmp[2];
    T T0[4], T1[4];
    T Gm[2] = {T(0), T(0)}, G0[2] = {T(0), T(0)};
    T Fm[9], F0[9];
    double UA[2], UB[2];
    T FA[9], FB[9];
    const T om = T(a.k.omega);
    T zero9[9];
#pragma unroll
    for (int q = 0; q < 9; q++) zero9[q] = T(0);

    // one iteration: consume the prefetched rows (u row r+3, populations row
    // r+1), refill the set with the rows of iteration r+2, update row r
    auto iteration = [&](int r, double Us[2], T Fs[9]) {
        double U3[2] = {Us[0], Us[1]};
        T F1[9];
#pragma unroll
        for (int q = 0; q < 9; q++) F1[q] = Fs[q];
        load_u(r + 5, Us);
        load_f(r + 3, Fs);
        T T2[4], G1[2];
        stress(r + 2, U1, U2, U3, T2);
        sigma(r + 1, T0, T1, T2, G1);

        // pull f(t_{r+1}) at row r: the forcing dt psi is added at the source node
        T h[9];
        h[0] = F0[0];
        h[1] = F0[1] + T(3) * wq<T>(1) * G0[0];
        h[3] = F0[3] - T(3) * wq<T>(3) * G0[0];
        h[2] = Fm[2] + T(3) * wq<T>(2) * Gm[1];
        h[5] = Fm[5] + T(3) * wq<T>(5) * (Gm[0] + Gm[1]);
        h[6] = Fm[6] + T(3) * wq<T>(6) * (Gm[1] - Gm[0]);
        h[4] = F1[4] - T(3) * wq<T>(4) * G1[1];
        h[7] = F1[7] - T(3) * wq<T>(7) * (G1[0] + G1[1]);
        h[8] = F1[8] + T(3) * wq<T>(8) * (G1[0] - G1[1]);
        T f[9];
        f[0] = h[0];
        f[1] = from_prev(h[1]);
        f[3] = from_next(h[3]);
        f[2] = h[2];
        f[5] = from_prev(h[5]);
        f[6] = from_next(h[6]);
        f[4] = h[4];
        f[7] = from_next(h[7]);
        f[8] = from_prev(h[8]);

        T rho = T(0), m1x = T(0), m1y = T(0), m2xx = T(0), m2xy = T(0), m2yy = T(0);
        T o1x = T(0), o1y = T(0);
#pragma unroll
        for (int q = 0; q < 9; q++) {
            rho += f[q];
            if (ex(q)) m1x += T(ex(q)) * f[q];
            if (ey(q)) m1y += T(ey(q)) * f[q];
            if (ex(q)) m2xx += f[q];
            if (ex(q) * ey(q)) m2xy += T(ex(q) * ey(q)) * f[q];
            if (ey(q)) m2yy += f[q];
            if (ex(q)) o1x += T(ex(q)) * F0[q];
            if (ey(q)) o1y += T(ey(q)) * F0[q];
        }
        const uint32_t node = (own && r >= yc && r < ye) ? (uint32_t)(r * g.pitch + x) : trash;
        T fn[9];
#pragma unroll
        for (int q = 0; q < 9; q++) {
            const T e = feq_q<T>(q, rho, m1x, m1y, m2xx, m2xy, m2yy);
            fn[q] = f[q] + om * (e - f[q]);
        }
        store_node(node, U0[0] + a.k.ucoef * (double)(m1x + o1x + G0[0]),
                   U0[1] + a.k.ucoef * (double)(m1y + o1y + G0[1]), fn);

        // rotate the computed rows
        U0[0] = U1[0]; U0[1] = U1[1];
        U1[0] = U2[0]; U1[1] = U2[1];
        U2[0] = U3[0]; U2[1] = U3[1];
#pragma unroll
        for (int c = 0; c < 4; c++) { T0[c] = T1[c]; T1[c] = T2[c]; }
        Gm[0] = G0[0]; Gm[1] = G0[1];
        G0[0] = G1[0]; G0[1] = G1[1];
#pragma unroll
        for (int q = 0; q < 9; q++) { Fm[q] = F0[q]; F0[q] = F1[q]; }
    };

    // prime the pipeline for the first iteration r = yc - 2; the prefetch sets
    // are loaded, each followed by the stores an iteration issues (to row ny),
    // so that the loop is entered with its memory operations in the same order
    // as from its back edge and the waits inside count alike on both paths
    load_u(yc - 3, tmp);
    load_u(yc - 2, U0);
    load_u(yc - 1, U1);
    load_u(yc, U2);
    load_u(yc + 1, UA);
    load_f(yc - 1, FA);
    store_node(trash, 0.0, 0.0, zero9);
    load_u(yc + 2, UB);
    load_f(yc, FB);
    store_node(trash, 0.0, 0.0, zero9);
    stress(yc - 2, tmp, U0, U1, T0);
    stress(yc - 1, U0, U1, U2, T1);
#pragma unroll
    for (int q = 0; q < 9; q++) { Fm[q] = T(0); F0[q] = T(0); }

    // an even number of iterations from yc - 2; one past ye only writes row ny
    for (int r = yc - 2; r < ye; r += 2) {
        iteration(r, UA, FA);
        iteration(r + 1, UB, FB);
    }
}

// ---- step: wall nodes ---------------------------------------------------------------------
//
// The nodes on non-periodic walls, one thread each, with global loads: the same
// stresses and sources as march_kernel (same expressions, same precision) and
// the wall rules of Sect. 3.3 for the links whose source lies beyond a wall.

// the i-th wall node: bottom row, top row, then the left and right columns
__device__ __forceinline__ bool wall_node(const Geometry& g, int i, int& x, int& y) {
    int k = i;
    if (!g.py) {
        if (k < g.nx) { x = k; y = 0; return true; }
        k -= g.nx;
        if (k < g.nx) { x = k; y = g.ny - 1; return true; }
        k -= g.nx;
    }
    if (!g.px) {
        const int y0 = g.py ? 0 : 1, nyi = g.py ? g.ny : g.ny - 2;
        if (k < nyi) { x = 0; y = y0 + k; return true; }
        k -= nyi;
        if (k < nyi) { x = g.nx - 1; y = y0 + k; return true; }
    }
    return false;
}

int wall_count(const Geometry& g) { return (g.py ? 0 : 2 * g.nx) + (g.px ? 0 : 2 * (g.py ? g.ny : g.ny - 2)); }

__device__ __forceinline__ double ld_uc(const StepArgs& a, int c, int x, int y) {
    return a.usrc[(size_t)c * a.g.plane + (size_t)y * a.g.pitch + x];
}

// T at an in-lattice node, as march_kernel's stress()
template <typename T, int MAT>
__device__ void wall_T(const StepArgs& a, int x, int y, T t[4]) {
    const Geometry& g = a.g;
    const double idx = a.k.inv_dx;
    int xl = x - 1, xr = x + 1, yl = y - 1, yr = y + 1;
    double fx = 0.5 * idx, fy = 0.5 * idx;
    if (g.px) { xl = wrap1(xl, g.nx); xr = wrap1(xr, g.nx); }
    else if (x == 0) { xl = x; fx = idx; }
    else if (x == g.nx - 1) { xr = x; fx = idx; }
    if (g.py) { yl = wrap1(yl, g.ny); yr = wrap1(yr, g.ny); }
    else if (y == 0) { yl = y; fy = idx; }
    else if (y == g.ny - 1) { yr = y; fy = idx; }
    excess_stress<T, MAT>(T((ld_uc(a, 0, xr, y) - ld_uc(a, 0, xl, y)) * fx),
                          T((ld_uc(a, 0, x, yr) - ld_uc(a, 0, x, yl)) * fy),
                          T((ld_uc(a, 1, xr, y) - ld_uc(a, 1, xl, y)) * fx),
                          T((ld_uc(a, 1, x, yr) - ld_uc(a, 1, x, yl)) * fy), T(a.k.lam), T(a.k.mu), t);
}

// sigma at an in-lattice node, as march_kernel's sigma()
template <typename T, int MAT>
__device__ void wall_sigma(const StepArgs& a, int x, int y, T sg[2]) {
    const Geometry& g = a.g;
    int xl = x - 1, xr = x + 1, yl = y - 1, yr = y + 1;
    T fx = T(0.5), fy = T(0.5);
    if (g.px) { xl = wrap1(xl, g.nx); xr = wrap1(xr, g.nx); }
    else if (x == 0) { xl = x; fx = T(1); }
    else if (x == g.nx - 1) { xr = x; fx = T(1); }
    if (g.py) { yl = wrap1(yl, g.ny); yr = wrap1(yr, g.ny); }
    else if (y == 0) { yl = y; fy = T(1); }
    else if (y == g.ny - 1) { yr = y; fy = T(1); }
    T tl[4], tr[4], tb[4], tt[4];
    wall_T<T, MAT>(a, xl, y, tl);
    wall_T<T, MAT>(a, xr, y, tr);
    wall_T<T, MAT>(a, x, yl, tb);
    wall_T<T, MAT>(a, x, yr, tt);
    sg[0] = T(a.k.inv_c2) * ((tr[0] - tl[0]) * fx + (tt[1] - tb[1]) * fy) + T(a.k.sig_b[0]);
    sg[1] = T(a.k.inv_c2) * ((tr[2] - tl[2]) * fx + (tt[3] - tb[3]) * fy) + T(a.k.sig_b[1]);
}

template <typename T, int MAT>
__global__ __launch_bounds__(256) void wall_kernel(StepArgs a, int nwall) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    int x, y;
    if (i >= nwall || !wall_node(a.g, i, x, y)) return;
    const Geometry g = a.g;
    const size_t plane = (size_t)g.plane;
    const size_t o = (size_t)y * g.pitch + x;
    const T* __restrict__ fs = reinterpret_cast<const T*>(a.fsrc);
    T* __restrict__ fd = reinterpret_cast<T*>(a.fdst);
    T fo[9];
#pragma unroll
    for (int q = 0; q < 9; q++) fo[q] = fs[q * plane + o];
    T G0[2], T0[4];
    wall_sigma<T, MAT>(a, x, y, G0);
    wall_T<T, MAT>(a, x, y, T0);
    const bool atL = at_low(x, g.px), atR = at_high(x, g.nx, g.px);
    const bool onB = at_low(y, g.py), onT = at_high(y, g.ny, g.py);

    // moments of the node's own populations at t_n (the collision keeps r and
    // Pi, and psi has no zeroth or second moment)
    double rr0 = 0, mxx = 0, myy = 0;
#pragma unroll
    for (int q = 0; q < 9; q++) {
        rr0 += (double)fo[q];
        mxx += (double)(ex(q) * ex(q)) * (double)fo[q];
        myy += (double)(ey(q) * ey(q)) * (double)fo[q];
    }
    const int wx = atL ? SIDE_L : SIDE_R, wy = onB ? SIDE_B : SIDE_T;
    const double sxw = atL ? -1.0 : 1.0, syw = onB ? -1.0 : 1.0;
    const double c2i = a.k.inv_c2;
    // Pi_bd / c^2 of the x wall and the y wall: normal row and column from the
    // traction balance, tangential entry from the node
    const double Xxx = (-sxw * a.w.val[wx][0] + (double)T0[0]) * c2i;
    const double Xxy = (-sxw * a.w.val[wx][1] + (double)T0[2]) * c2i;
    const double Yyy = (-syw * a.w.val[wy][1] + (double)T0[3]) * c2i;
    const double Yxy = (-syw * a.w.val[wy][0] + (double)T0[1]) * c2i;

    T f[9];
#pragma unroll
    for (int p = 0; p < 9; p++) {
        int sxp = x - ex(p), syp = y - ey(p);
        bool crx = false, cry = false;
        if (g.px) sxp = wrap1(sxp, g.nx); else crx = sxp < 0 || sxp >= g.nx;
        if (g.py) syp = wrap1(syp, g.ny); else cry = syp < 0 || syp >= g.ny;
        if (!crx && !cry) {
            T gs[2] = {G0[0], G0[1]};
            if (p != 0) wall_sigma<T, MAT>(a, sxp, syp, gs);
            f[p] = fs[p * plane + (size_t)syp * g.pitch + sxp] +
                   T(3) * wq<T>(p) * (T(ex(p)) * gs[0] + T(ey(p)) * gs[1]);
            continue;
        }
        const int q = opp(p);  // the outgoing link the wall reflects
        const double fcq = (double)fo[q] + 3.0 * wq<double>(q) *
                           ((double)ex(q) * (double)G0[0] + (double)ey(q) * (double)G0[1]);
        double jx = 0.0, jy = 0.0;
        int nd = 0;
        if (crx && a.w.bc[wx] == BC_DIR) { jx += a.w.val[wx][0]; jy += a.w.val[wx][1]; nd++; }
        if (cry && a.w.bc[wy] == BC_DIR) { jx += a.w.val[wy][0]; jy += a.w.val[wy][1]; nd++; }
        double v;
        if (nd > 0) {
            // modified bounce-back, Eq. bbcon: -(2/cs^2) w c.j* = -6 w e.(j*/c)
            const double sc = a.k.inv_c / (double)nd;
            v = fcq - 6.0 * wq<double>(q) * ((double)ex(q) * jx + (double)ey(q) * jy) * sc;
        } else {
            // modified anti-bounce-back, Eq. abbcon
            double Mxx, Mxy, Myy;
            if (crx && cry) { Mxx = Xxx; Myy = Yyy; Mxy = 0.5 * (Xxy + Yxy); }
            else if (crx) { Mxx = Xxx; Mxy = Xxy; Myy = myy; }
            else { Mxx = mxx; Mxy = Yxy; Myy = Yyy; }
            const double X = ex(q), Y = ey(q);
            const double eMe = X * X * Mxx + 2.0 * X * Y * Mxy + Y * Y * Myy;
            const double e2 = X * X + Y * Y;
            v = -fcq + 2.0 * wq<double>(q) * (rr0 + 0.5 * (9.0 * eMe - 3.0 * rr0 * e2 - 3.0 * (Mxx + Myy) + 2.0 * rr0));
        }
        f[p] = T(v);
    }

    T rho = T(0), m1x = T(0), m1y = T(0), m2xx = T(0), m2xy = T(0), m2yy = T(0);
    T o1x = T(0), o1y = T(0);
#pragma unroll
    for (int q = 0; q < 9; q++) {
        rho += f[q];
        if (ex(q)) m1x += T(ex(q)) * f[q];
        if (ey(q)) m1y += T(ey(q)) * f[q];
        if (ex(q)) m2xx += f[q];
        if (ex(q) * ey(q)) m2xy += T(ex(q) * ey(q)) * f[q];
        if (ey(q)) m2yy += f[q];
        if (ex(q)) o1x += T(ex(q)) * fo[q];
        if (ey(q)) o1y += T(ey(q)) * fo[q];
    }
    a.udst[o] = a.usrc[o] + a.k.ucoef * (double)(m1x + o1x + G0[0]);
    a.udst[plane + o] = a.usrc[plane + o] + a.k.ucoef * (double)(m1y + o1y + G0[1]);
    const T om = T(a.k.omega);
#pragma unroll
    for (int q = 0; q < 9; q++) {
        const T e = feq_q<T>(q, rho, m1x, m1y, m2xx, m2xy, m2yy);
        fd[q * plane + o] = f[q] + om * (e - f[q]);
    }
}

// ---- per-node helpers for init, read-out and diagnostics (FP64, global loads) ----------

__device__ __forceinline__ double ld_u(const InitLike& a, int c, int gx, int gy) {
    return a.u[(size_t)c * a.g.plane + (size_t)gy * a.g.pitch + gx];
}

// H = grad u at a node, (xx, xy, yx, yy)
__device__ void node_H(const InitLike& a, int gx, int gy, double H[4]) {
    const Geometry& g = a.g;
    int xl = gx - 1, xr = gx + 1, yl = gy - 1, yr = gy + 1;
    double fx = 0.5 * a.inv_dx, fy = 0.5 * a.inv_dx;
    if (g.px) { xl = wrap1(xl, g.nx); xr = wrap1(xr, g.nx); }
    else if (gx == 0) { xl = gx; fx = a.inv_dx; }
    else if (gx == g.nx - 1) { xr = gx; fx = a.inv_dx; }
    if (g.py) { yl = wrap1(yl, g.ny); yr = wrap1(yr, g.ny); }
    else if (gy == 0) { yl = gy; fy = a.inv_dx; }
    else if (gy == g.ny - 1) { yr = gy; fy = a.inv_dx; }
    H[0] = (ld_u(a, 0, xr, gy) - ld_u(a, 0, xl, gy)) * fx;
    H[1] = (ld_u(a, 0, gx, yr) - ld_u(a, 0, gx, yl)) * fy;
    H[2] = (ld_u(a, 1, xr, gy) - ld_u(a, 1, xl, gy)) * fx;
    H[3] = (ld_u(a, 1, gx, yr) - ld_u(a, 1, gx, yl)) * fy;
}

template <int MAT>
__device__ void node_T(const InitLike& a, int gx, int gy, double t[4]) {
    double H[4];
    node_H(a, gx, gy, H);
    excess_stress<double, MAT>(H[0], H[1], H[2], H[3], a.lam, a.mu, t);
}

// sigma = dt S / c at a node
template <int MAT>
__device__ void node_sigma(const InitLike& a, int gx, int gy, double s[2]) {
    const Geometry& g = a.g;
    int xl = gx - 1, xr = gx + 1, yl = gy - 1, yr = gy + 1;
    double fx = 0.5, fy = 0.5;
    if (g.px) { xl = wrap1(xl, g.nx); xr = wrap1(xr, g.nx); }
    else if (gx == 0) { xl = gx; fx = 1.0; }
    else if (gx == g.nx - 1) { xr = gx; fx = 1.0; }
    if (g.py) { yl = wrap1(yl, g.ny); yr = wrap1(yr, g.ny); }
    else if (gy == 0) { yl = gy; fy = 1.0; }
    else if (gy == g.ny - 1) { yr = gy; fy = 1.0; }
    double tl[4], tr[4], tb[4], tt[4];
    node_T<MAT>(a, xl, gy, tl);
    node_T<MAT>(a, xr, gy, tr);
    node_T<MAT>(a, gx, yl, tb);
    node_T<MAT>(a, gx, yr, tt);
    s[0] = a.inv_c2 * ((tr[0] - tl[0]) * fx + (tt[1] - tb[1]) * fy) + a.sig_b[0];
    s[1] = a.inv_c2 * ((tr[2] - tl[2]) * fx + (tt[3] - tb[3]) * fy) + a.sig_b[1];
}

// ---- init ------------------------------------------------------------------------------

// fc'_0 = f_eq(r0 = -rho0 tr H(u0), j0, Pi(H(u0))): an equilibrium is unchanged by
// the collision without forcing.
template <typename T>
__global__ __launch_bounds__(256) void init_kernel(InitArgs a) {
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (gx >= a.b.g.nx || gy >= a.b.g.ny) return;
    const size_t plane = (size_t)a.b.g.plane;
    const size_t o = (size_t)gy * a.b.g.pitch + gx;
    double H[4];
    node_H(a.b, gx, gy, H);
    const double tr = H[0] + H[3];
    const double r0 = -a.rho0 * tr;
    const double ic2 = a.b.inv_c2;
    const double m2xx = -a.b.mu * (H[0] + H[0] + tr) * ic2;
    const double m2xy = -a.b.mu * (H[1] + H[2]) * ic2;
    const double m2yy = -a.b.mu * (H[3] + H[3] + tr) * ic2;
    const double m1x = a.j0[o] * a.inv_c, m1y = a.j0[plane + o] * a.inv_c;
    T* f = reinterpret_cast<T*>(a.f);
#pragma unroll
    for (int q = 0; q < 9; q++)
        f[q * plane + o] = T(feq_q<double>(q, r0, m1x, m1y, m2xx, m2xy, m2yy));
}

// ---- read-out -----------------------------------------------------------------------------

template <typename T, int MAT>
__global__ __launch_bounds__(256) void read_kernel(ReadArgs a) {
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    const Geometry& g = a.b.g;
    if (gx >= g.nx || gy >= g.ny) return;
    const size_t plane = (size_t)g.plane;
    const size_t o = (size_t)gy * g.pitch + gx;
    const size_t oc = (size_t)gy * g.nx + gx, pc = (size_t)g.nx * g.ny;  // compact output
    const T* fs = reinterpret_cast<const T*>(a.f);
    double* d = a.dst;
    switch (a.field) {
    case 0:  // U
        d[oc] = a.b.u[o];
        d[pc + oc] = a.b.u[plane + o];
        break;
    case 1: {  // J = c (M1' + sigma / 2)
        double s[2], mx = 0, my = 0;
        node_sigma<MAT>(a.b, gx, gy, s);
        for (int q = 0; q < 9; q++) {
            const double v = (double)fs[q * plane + o];
            mx += ex(q) * v;
            my += ey(q) * v;
        }
        d[oc] = a.c * (mx + 0.5 * s[0]);
        d[pc + oc] = a.c * (my + 0.5 * s[1]);
        break;
    }
    case 2:  // R
    case 3: {  // PI = c^2 M2'
        double r = 0, pxx = 0, pxy = 0, pyy = 0;
        for (int q = 0; q < 9; q++) {
            const double v = (double)fs[q * plane + o];
            r += v;
            pxx += ex(q) * ex(q) * v;
            pxy += ex(q) * ey(q) * v;
            pyy += ey(q) * ey(q) * v;
        }
        if (a.field == 2) {
            d[oc] = r;
        } else {
            const double c2 = a.c * a.c;
            d[oc] = c2 * pxx;
            d[pc + oc] = c2 * pxy;
            d[2 * pc + oc] = c2 * pyy;
        }
        break;
    }
    case 4:  // H
    case 5: {  // P
        double H[4], P[4];
        node_H(a.b, gx, gy, H);
        if (a.field == 5) first_pk<double, MAT>(H[0], H[1], H[2], H[3], a.b.lam, a.b.mu, P);
        for (int c = 0; c < 4; c++) d[c * pc + oc] = a.field == 4 ? H[c] : P[c];
        break;
    }
    case 6: {  // S
        double s[2];
        node_sigma<MAT>(a.b, gx, gy, s);
        d[oc] = s[0] * a.s_from_sig;
        d[pc + oc] = s[1] * a.s_from_sig;
        break;
    }
    default: break;
    }
}

// ---- diagnostics: fixed-order block reductions ------------------------------------------------

template <typename T, int MAT>
__global__ __launch_bounds__(256) void diag_kernel(ReadArgs a) {
    const Geometry& g = a.b.g;
    const int nbx = (g.nx + 63) / 64;
    const int bx = blockIdx.x % nbx, by = blockIdx.x / nbx;
    const int gx = bx * 64 + (threadIdx.x & 63), gy = by * 4 + (threadIdx.x >> 6);
    double v[5] = {0, 0, 0, 0, 0};  // momentum x, y, ekin, max |u|^2, non-finite
    if (gx < g.nx && gy < g.ny) {
        const size_t plane = (size_t)g.plane;
        const size_t o = (size_t)gy * g.pitch + gx;
        const T* fs = reinterpret_cast<const T*>(a.f);
        double mx = 0, my = 0, s[2];
        for (int q = 0; q < 9; q++) {
            const double w = (double)fs[q * plane + o];
            mx += ex(q) * w;
            my += ey(q) * w;
        }
        node_sigma<MAT>(a.b, gx, gy, s);
        const double jx = a.c * (mx + 0.5 * s[0]), jy = a.c * (my + 0.5 * s[1]);
        const double ux = a.b.u[o], uy = a.b.u[plane + o];
        v[0] = a.c * mx;
        v[1] = a.c * my;
        v[2] = (jx * jx + jy * jy) / (2.0 * a.b.rho0);
        v[3] = ux * ux + uy * uy;
        v[4] = (isfinite(jx) && isfinite(jy) && isfinite(ux) && isfinite(uy)) ? 0.0 : 1.0;
        if (v[4] != 0.0) v[3] = 0.0;
    }
    __shared__ double red[5][256];
    for (int c = 0; c < 5; c++) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int c = 0; c < 5; c++) {
                const double x = red[c][threadIdx.x], y = red[c][threadIdx.x + w];
                red[c][threadIdx.x] = (c == 3 || c == 4) ? fmax(x, y) : x + y;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) a.partial[(size_t)blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void diag_reduce_kernel(double* partial, int nblk, double* out) {
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256)
        for (int c = 0; c < 5; c++) {
            const double x = partial[(size_t)b * 8 + c];
            v[c] = (c == 3 || c == 4) ? fmax(v[c], x) : v[c] + x;
        }
    __shared__ double red[5][256];
    for (int c = 0; c < 5; c++) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 5; c++) {
                const double x = red[c][threadIdx.x], y = red[c][threadIdx.x + w];
                red[c][threadIdx.x] = (c == 3 || c == 4) ? fmax(x, y) : x + y;
            }
        __syncthreads();
    }
    if (threadIdx.x < 5) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---- launchers ---------------------------------------------------------------------------------

// rows per chunk of the marching kernel: enough waves to fill the chip twice
// over, without letting the rows that prime each chunk dominate
static int march_chunk(const Geometry& g, int nstrip) {
    const long target = 16384;
    long c = ((long)g.ny * nstrip + target - 1) / target;
    c = c < 8 ? 8 : (c > 128 ? 128 : c);
    return (int)c;
}

template <typename T, int MAT>
static void step_m(const StepArgs& a, hipStream_t st) {
    const int nstrip = (a.g.nx + MO - 1) / MO;
    const int chunk = march_chunk(a.g, nstrip);
    const int nchunk = (a.g.ny + chunk - 1) / chunk;
    hipLaunchKernelGGL((march_kernel<T, MAT>), dim3((nstrip * nchunk + 3) / 4), dim3(256), 0, st, a, nstrip,
                       nchunk, chunk);
    const int nwall = wall_count(a.g);
    if (nwall > 0)
        hipLaunchKernelGGL((wall_kernel<T, MAT>), dim3((nwall + 255) / 256), dim3(256), 0, st, a, nwall);
}

template <typename T>
static hipError_t step_t(int material, const StepArgs& a, hipStream_t st) {
    switch (material) {
    case MAT_SVK: step_m<T, MAT_SVK>(a, st); break;
    case MAT_NH: step_m<T, MAT_NH>(a, st); break;
    default: step_m<T, MAT_LIN>(a, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_step(int f64, int material, const StepArgs& a, hipStream_t st) {
    return f64 ? step_t<double>(material, a, st) : step_t<float>(material, a, st);
}

hipError_t launch_init(int f64, const InitArgs& a, hipStream_t st) {
    const dim3 grid((a.b.g.nx + 63) / 64, (a.b.g.ny + 3) / 4), block(256);
    if (f64) hipLaunchKernelGGL((init_kernel<double>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((init_kernel<float>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t read_t(int material, const ReadArgs& a, hipStream_t st) {
    const dim3 grid((a.b.g.nx + 63) / 64, (a.b.g.ny + 3) / 4), block(256);
    switch (material) {
    case MAT_SVK: hipLaunchKernelGGL((read_kernel<T, MAT_SVK>), grid, block, 0, st, a); break;
    case MAT_NH: hipLaunchKernelGGL((read_kernel<T, MAT_NH>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((read_kernel<T, MAT_LIN>), grid, block, 0, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_read(int f64, int material, const ReadArgs& a, hipStream_t st) {
    return f64 ? read_t<double>(material, a, st) : read_t<float>(material, a, st);
}

int diag_blocks(const Geometry& g) { return ((g.nx + 63) / 64) * ((g.ny + 3) / 4); }

template <typename T>
static hipError_t diag_t(int material, const ReadArgs& a, double* out, hipStream_t st) {
    const int nblk = diag_blocks(a.b.g);
    switch (material) {
    case MAT_SVK: hipLaunchKernelGGL((diag_kernel<T, MAT_SVK>), dim3(nblk), dim3(256), 0, st, a); break;
    case MAT_NH: hipLaunchKernelGGL((diag_kernel<T, MAT_NH>), dim3(nblk), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((diag_kernel<T, MAT_LIN>), dim3(nblk), dim3(256), 0, st, a); break;
    }
    hipLaunchKernelGGL(diag_reduce_kernel, dim3(1), dim3(256), 0, st, a.partial, nblk, out);
    return hipGetLastError();
}

hipError_t launch_diag(int f64, int material, const ReadArgs& a, double* out, hipStream_t st) {
    return f64 ? diag_t<double>(material, a, out, st) : diag_t<float>(material, a, out, st);
}

}  // namespace mclbm
