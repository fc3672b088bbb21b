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
// (one pass over HBM, each wave owning 64 aligned columns of a band of rows),
// then wall_kernel recomputes the nodes on non-periodic walls (0.05 % of an
// 8192^2 lattice) with the wall rules.
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

template <typename V>
__device__ __forceinline__ V from_prev(V v) { return __shfl_up(v, 1); }    // value of lane l-1
template <typename V>
__device__ __forceinline__ V from_next(V v) { return __shfl_down(v, 1); }  // value of lane l+1

// ---- step: interior nodes, y-marching ------------------------------------------------------
//
// Each wave owns the 64 columns [64 s, 64 s + 64) of a strip, so that every
// store covers whole cache lines (a partly written line costs a read-modify-
// write in HBM).  The values lanes 0 and 63 need from the neighbouring columns
// (u of x0-1 and x0+64, their T, and the pulled populations with their forcing)
// come from a halo pass every HR rows: it gathers u on five columns per side,
// computes T on three and sigma and the six pull sources on the neighbour
// column, and leaves them in wave-private LDS (no barrier: only this wave reads
// them).  The gathers of a halo pass are issued one block ahead.  Lanes beyond
// nx compute on clamped (or, periodic, wrapped) data and store into the row
// padding; rows that prime the pipeline store into row ny.

constexpr int HR = 6;       // iterations per halo block
constexpr int HK = HR + 6;  // halo rows per block: k = 0..HK-1 is row r0 - 3 + k

template <typename T>
struct Halo {
    double u[2][HK][5][2];  // [side][k][column c][comp]; side 0: x0-3+c, side 1: x0+62+c
    T t[2][HK][3][4];       // T at c = 1, 2, 3
    T s[2][HK][2];          // sigma at c = 2
    T h[2][HK][3];          // pull sources at c = 2: side 0 p = 1, 5, 8; side 1 p = 3, 6, 7
};

// orders this wave's LDS writes before its later reads by other lanes (the
// LDS serves one wave's operations in issue order; this keeps the compiler's
// order too)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int halo_pop(int side, int i) {
    return side == 0 ? (i == 0 ? 1 : (i == 1 ? 5 : 8)) : (i == 0 ? 3 : (i == 1 ? 6 : 7));
}

template <typename T, int MAT>
__global__ __launch_bounds__(256) void march_kernel(StepArgs a, int nstrip, int nchunk, int chunk) {
    __shared__ Halo<T> halo_lds[4];
    const Geometry g = a.g;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    Halo<T>& hl = halo_lds[wv];
    const int item = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + wv);
    if (item >= nstrip * nchunk) return;
    const int strip = item % nstrip, chk = item / nstrip;
    const int x0 = strip * 64;
    const int vx = x0 + lane;  // this lane's column (< pitch)
    // column -> column to address: periodic wrap, else clamped into the lattice
    auto colp = [&](int c) -> int { return g.px ? wrap(c, g.nx) : min(max(c, 0), g.nx - 1); };
    const int x = colp(vx);
    const bool xin = g.px ? true : vx < g.nx;
    const bool atL = xin && at_low(x, g.px), atR = xin && at_high(x, g.nx, g.px);
    const int yc = chk * chunk, ye = min(yc + chunk, g.ny);
    const int nblk = (ye - (yc - 2) + HR - 1) / HR;
    const size_t plane = (size_t)g.plane;
    const uint32_t pbT = (uint32_t)(plane * sizeof(T)), pbD = (uint32_t)(plane * sizeof(double));
    const T* fs = reinterpret_cast<const T*>(a.fsrc);
    T* fd = reinterpret_cast<T*>(a.fdst);
    const __amdgpu_buffer_rsrc_t rs0 = rsrc(fs, 3 * pbT), rs1 = rsrc(fs + 3 * plane, 3 * pbT),
                                 rs2 = rsrc(fs + 6 * plane, 3 * pbT);
    const __amdgpu_buffer_rsrc_t rd0 = rsrc(fd, 3 * pbT), rd1 = rsrc(fd + 3 * plane, 3 * pbT),
                                 rd2 = rsrc(fd + 6 * plane, 3 * pbT);
    const __amdgpu_buffer_rsrc_t rus = rsrc(a.usrc, 2 * pbD), rud = rsrc(a.udst, 2 * pbD);
    const double idx = a.k.inv_dx;
    const T ic2 = T(a.k.inv_c2), sbx = T(a.k.sig_b[0]), sby = T(a.k.sig_b[1]);
    const T lam = T(a.k.lam), mu = T(a.k.mu);
    const uint32_t trash = (uint32_t)(g.ny * g.pitch + vx);  // row ny: written, never read

    // row r -> row to address (periodic wrap, else clamped)
    auto rowp = [&](int r) -> int { return g.py ? wrap(r, g.ny) : min(max(r, 0), g.ny - 1); };
    auto load_u = [&](int r, double v[2]) {
        const uint32_t ob = (uint32_t)(rowp(r) * g.pitch + x) * (uint32_t)sizeof(double);
        v[0] = bload(rus, ob, 0u, 0.0);
        v[1] = bload(rus, ob, pbD, 0.0);
    };
    auto load_f = [&](int r, T f[9]) {
        const uint32_t ob = (uint32_t)(rowp(r) * g.pitch + x) * (uint32_t)sizeof(T);
#pragma unroll
        for (int q = 0; q < 9; q++)
            f[q] = bload(q < 3 ? rs0 : (q < 6 ? rs1 : rs2), ob, (uint32_t)(q % 3) * pbT, T(0));
    };
    auto store_node = [&](uint32_t node, double ux, double uy, const T fn[9]) {
        const uint32_t ou = node * (uint32_t)sizeof(double), of = node * (uint32_t)sizeof(T);
        bstore(rud, ou, 0u, ux);
        bstore(rud, ou, pbD, uy);
#pragma unroll
        for (int q = 0; q < 9; q++)
            bstore(q < 3 ? rd0 : (q < 6 ? rd1 : rd2), of, (uint32_t)(q % 3) * pbT, fn[q]);
    };
    // one-sided differences at the lattice edges, central elsewhere
    auto lo_row = [&](int r) { return !g.py && rowp(r) == 0 && r <= 0; };
    auto hi_row = [&](int r) { return !g.py && rowp(r) == g.ny - 1 && r >= g.ny - 1; };

    // T = P(H) + Pi(H) at row r of this lane; pl*/pr* replace the u of the
    // column left of lane 0 / right of lane 63
    auto stress = [&](int r, const double um[2], const double u0[2], const double up[2], T t[4], double plx,
                      double ply, double prx, double pry) {
        double lx = from_prev(u0[0]), rx = from_next(u0[0]);
        double ly = from_prev(u0[1]), ry = from_next(u0[1]);
        lx = lane == 0 ? plx : lx;
        ly = lane == 0 ? ply : ly;
        rx = lane == 63 ? prx : rx;
        ry = lane == 63 ? pry : ry;
        const double ax = atL ? u0[0] : lx, bx = atR ? u0[0] : rx;
        const double ay = atL ? u0[1] : ly, by = atR ? u0[1] : ry;
        const double fx = (atL || atR) ? idx : 0.5 * idx;
        const bool lo = lo_row(r), hi = hi_row(r);
        const double cx = lo ? u0[0] : um[0], dx = hi ? u0[0] : up[0];
        const double cy = lo ? u0[1] : um[1], dy = hi ? u0[1] : up[1];
        const double fy = (lo || hi) ? idx : 0.5 * idx;
        excess_stress<T, MAT>(T((bx - ax) * fx), T((dx - cx) * fy), T((by - ay) * fx), T((dy - cy) * fy),
                              lam, mu, t);
    };
    // sigma = dt S / c at row r of this lane; pl*/pr* replace T_xx, T_yx of the
    // column left of lane 0 / right of lane 63
    auto sigma = [&](int r, const T tm[4], const T t0[4], const T tp[4], T sg[2], T plxx, T plyx, T prxx,
                     T pryx) {
        T lxx = from_prev(t0[0]), rxx = from_next(t0[0]);
        T lyx = from_prev(t0[2]), ryx = from_next(t0[2]);
        lxx = lane == 0 ? plxx : lxx;
        lyx = lane == 0 ? plyx : lyx;
        rxx = lane == 63 ? prxx : rxx;
        ryx = lane == 63 ? pryx : ryx;
        const T axx = atL ? t0[0] : lxx, bxx = atR ? t0[0] : rxx;
        const T ayx = atL ? t0[2] : lyx, byx = atR ? t0[2] : ryx;
        const T fx = (atL || atR) ? T(1) : T(0.5);
        const bool lo = lo_row(r), hi = hi_row(r);
        const T cxy = lo ? t0[1] : tm[1], dxy = hi ? t0[1] : tp[1];
        const T cyy = lo ? t0[3] : tm[3], dyy = hi ? t0[3] : tp[3];
        const T fy = (lo || hi) ? T(1) : T(0.5);
        sg[0] = ic2 * ((bxx - axx) * fx + (dxy - cxy) * fy) + sbx;
        sg[1] = ic2 * ((byx - ayx) * fx + (dyy - cyy) * fy) + sby;
    };

    // ---- halo: gathers (issued one block ahead) and the pass that fills the LDS
    double gux[2], guy[2];
    T gf;
    auto gather = [&](int r0) {
        const int i = min(lane, 5 * HK - 1);
        const int c = i % 5, k = i / 5;
        const int rr = rowp(r0 - 3 + k);
#pragma unroll
        for (int sd = 0; sd < 2; sd++) {
            const int hx = colp(sd == 0 ? x0 - 3 + c : x0 + 62 + c);
            const uint32_t ob = (uint32_t)(rr * g.pitch + hx) * (uint32_t)sizeof(double);
            gux[sd] = bload(rus, ob, 0u, 0.0);
            guy[sd] = bload(rus, ob, pbD, 0.0);
        }
        const int j = min(lane, 47);
        const int sd = j / 24, pi = (j % 24) / 8, k2 = 2 + j % 8;
        const int hx = colp(sd == 0 ? x0 - 1 : x0 + 64);
        gf = fs[(size_t)halo_pop(sd, pi) * plane + (size_t)rowp(r0 - 3 + k2) * g.pitch + hx];
    };
    auto halo = [&](int r0) {
        wave_lds_sync();  // the last block's reads come first
        if (lane < 5 * HK) {
            const int c = lane % 5, k = lane / 5;
#pragma unroll
            for (int sd = 0; sd < 2; sd++) {
                hl.u[sd][k][c][0] = gux[sd];
                hl.u[sd][k][c][1] = guy[sd];
            }
        }
        wave_lds_sync();
        if (lane < 60) {  // T at c = 1, 2, 3 and k = 1..10, both sides
            const int sd = lane / 30, jj = lane % 30, c = 1 + jj % 3, k = 1 + jj / 3;
            const int X = colp(sd == 0 ? x0 - 3 + c : x0 + 62 + c);
            const int r = r0 - 3 + k;
            const double u0x = hl.u[sd][k][c][0], u0y = hl.u[sd][k][c][1];
            const bool aL = !g.px && X == 0, aR = !g.px && X == g.nx - 1;
            const double ax = aL ? u0x : hl.u[sd][k][c - 1][0], bx = aR ? u0x : hl.u[sd][k][c + 1][0];
            const double ay = aL ? u0y : hl.u[sd][k][c - 1][1], by = aR ? u0y : hl.u[sd][k][c + 1][1];
            const double fx = (aL || aR) ? idx : 0.5 * idx;
            const bool lo = lo_row(r), hi = hi_row(r);
            const double cx = lo ? u0x : hl.u[sd][k - 1][c][0], dx = hi ? u0x : hl.u[sd][k + 1][c][0];
            const double cy = lo ? u0y : hl.u[sd][k - 1][c][1], dy = hi ? u0y : hl.u[sd][k + 1][c][1];
            const double fy = (lo || hi) ? idx : 0.5 * idx;
            T t[4];
            excess_stress<T, MAT>(T((bx - ax) * fx), T((dx - cx) * fy), T((by - ay) * fx), T((dy - cy) * fy),
                                  lam, mu, t);
#pragma unroll
            for (int q = 0; q < 4; q++) hl.t[sd][k][c - 1][q] = t[q];
        }
        wave_lds_sync();
        if (lane < 16) {  // sigma at c = 2 and k = 2..9
            const int sd = lane / 8, k = 2 + lane % 8;
            const int X = colp(sd == 0 ? x0 - 1 : x0 + 64);
            const int r = r0 - 3 + k;
            const bool aL = !g.px && X == 0, aR = !g.px && X == g.nx - 1;
            const T t0xx = hl.t[sd][k][1][0], t0yx = hl.t[sd][k][1][2];
            const T axx = aL ? t0xx : hl.t[sd][k][0][0], bxx = aR ? t0xx : hl.t[sd][k][2][0];
            const T ayx = aL ? t0yx : hl.t[sd][k][0][2], byx = aR ? t0yx : hl.t[sd][k][2][2];
            const T fx = (aL || aR) ? T(1) : T(0.5);
            const bool lo = lo_row(r), hi = hi_row(r);
            const T cxy = lo ? hl.t[sd][k][1][1] : hl.t[sd][k - 1][1][1];
            const T dxy = hi ? hl.t[sd][k][1][1] : hl.t[sd][k + 1][1][1];
            const T cyy = lo ? hl.t[sd][k][1][3] : hl.t[sd][k - 1][1][3];
            const T dyy = hi ? hl.t[sd][k][1][3] : hl.t[sd][k + 1][1][3];
            const T fy = (lo || hi) ? T(1) : T(0.5);
            hl.s[sd][k][0] = ic2 * ((bxx - axx) * fx + (dxy - cxy) * fy) + sbx;
            hl.s[sd][k][1] = ic2 * ((byx - ayx) * fx + (dyy - cyy) * fy) + sby;
        }
        wave_lds_sync();
        if (lane < 48) {  // pull sources: the population plus dt psi at the source
            const int sd = lane / 24, pi = (lane % 24) / 8, k = 2 + lane % 8;
            const int p = halo_pop(sd, pi);
            hl.h[sd][k][pi] = gf + T(3) * wq<T>(p) * (T(ex(p)) * hl.s[sd][k][0] + T(ey(p)) * hl.s[sd][k][1]);
        }
        wave_lds_sync();
    };

    // ---- the row pipeline
    // At iteration r the wave holds in registers the rows r..r+3 of u, r..r+2 of
    // T, r-1..r+1 of sigma and r-1..r+1 of the populations, and the loads of the
    // rows two iterations ahead are in flight (two prefetch sets A and B, so that
    // no register holding a pending load is renamed).  x neighbours come from
    // lane shuffles, y neighbours from the rows held; every iteration issues the
    // same loads and stores in the same order, so the waits stay counted.
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

    // iteration r of the block's relative row rel (0..HR-1)
    auto iteration = [&](int r, int rel, double Us[2], T Fs[9]) {
        double U3[2] = {Us[0], Us[1]};
        T F1[9];
#pragma unroll
        for (int q = 0; q < 9; q++) F1[q] = Fs[q];
        load_u(r + 5, Us);
        load_f(r + 3, Fs);
        T T2[4], G1[2];
        stress(r + 2, U1, U2, U3, T2, hl.u[0][rel + 5][2][0], hl.u[0][rel + 5][2][1], hl.u[1][rel + 5][2][0],
               hl.u[1][rel + 5][2][1]);
        sigma(r + 1, T0, T1, T2, G1, hl.t[0][rel + 4][1][0], hl.t[0][rel + 4][1][2], hl.t[1][rel + 4][1][0],
              hl.t[1][rel + 4][1][2]);

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
        f[2] = h[2];
        f[4] = h[4];
        {
            const T f1 = from_prev(h[1]), f5 = from_prev(h[5]), f8 = from_prev(h[8]);
            const T f3 = from_next(h[3]), f6 = from_next(h[6]), f7 = from_next(h[7]);
            f[1] = lane == 0 ? hl.h[0][rel + 3][0] : f1;
            f[5] = lane == 0 ? hl.h[0][rel + 2][1] : f5;
            f[8] = lane == 0 ? hl.h[0][rel + 4][2] : f8;
            f[3] = lane == 63 ? hl.h[1][rel + 3][0] : f3;
            f[6] = lane == 63 ? hl.h[1][rel + 2][1] : f6;
            f[7] = lane == 63 ? hl.h[1][rel + 4][2] : f7;
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
            if (ex(q)) o1x += T(ex(q)) * F0[q];
            if (ey(q)) o1y += T(ey(q)) * F0[q];
        }
        const uint32_t node = (r >= yc && r < ye) ? (uint32_t)(r * g.pitch + vx) : trash;
        T fn[9];
#pragma unroll
        for (int q = 0; q < 9; q++) {
            const T e = feq_q<T>(q, rho, m1x, m1y, m2xx, m2xy, m2yy);
            fn[q] = f[q] + om * (e - f[q]);
        }
        store_node(node, U0[0] + a.k.ucoef * (double)(m1x + o1x + G0[0]),
                   U0[1] + a.k.ucoef * (double)(m1y + o1y + G0[1]), fn);

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

    // prime: the halo of the first block (waited for here, once per chunk), the
    // rows, the two prefetch sets each followed by the stores an iteration issues,
    // and the gathers of the next block, in the order the loop repeats
    int r0 = yc - 2;
    gather(r0);
    halo(r0);
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
    gather(r0 + HR);
    stress(yc - 2, tmp, U0, U1, T0, hl.u[0][3][2][0], hl.u[0][3][2][1], hl.u[1][3][2][0], hl.u[1][3][2][1]);
    stress(yc - 1, U0, U1, U2, T1, hl.u[0][4][2][0], hl.u[0][4][2][1], hl.u[1][4][2][0], hl.u[1][4][2][1]);
#pragma unroll
    for (int q = 0; q < 9; q++) { Fm[q] = T(0); F0[q] = T(0); }

    for (int b = 0; b < nblk; b++) {
        iteration(r0 + 0, 0, UA, FA);
        iteration(r0 + 1, 1, UB, FB);
        iteration(r0 + 2, 2, UA, FA);
        iteration(r0 + 3, 3, UB, FB);
        iteration(r0 + 4, 4, UA, FA);
        iteration(r0 + 5, 5, UB, FB);
        r0 += HR;
        halo(r0);
        gather(r0 + HR);
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

// rows per chunk of march_kernel: a multiple of HR minus the two priming
// rows, with enough waves to fill the chip twice over
static int march_chunk(const Geometry& g, int nstrip) {
    const long target = 16384;
    long c = ((long)g.ny * nstrip + target - 1) / target;
    long m = (c + 2 + HR - 1) / HR;
    if (m < 1) m = 1;
    if (m * HR - 2 > 190) m = (190 + 2) / HR;
    return (int)(m * HR - 2);
}

template <typename T, int MAT>
static void step_m(const StepArgs& a, hipStream_t st) {
    const int nstrip = a.g.pitch / 64;
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
