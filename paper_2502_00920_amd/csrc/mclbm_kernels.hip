// HIP kernels of the moment-chain LBM step for gfx950 (MI355X).
//
// One time step of Algorithm 1 (with the stresses taken at the current level,
// Sect. 3.1) is one launch of step_kernel.  The state between launches is
//   fc' = the post-collision populations WITHOUT the forcing term, and u (FP64).
// This works because the forcing enters the BGK collision additively:
//   f - (f - f_eq(r, j, Pi))/tau* + (1 - 1/(2 tau*)) psi(S) dt
//     = (1 - 1/tau*) f + f_eq(r, sum c f, Pi)/tau* + dt psi(S)
// (j = sum c f + dt/2 S enters f_eq linearly), so the launch for step n can add
// dt psi(S_n) while it pulls the populations, once S_n is known from u_n.
//
// Launch for step n, per tile of TX x TY nodes:
//   1. u_n on the tile and a halo of 3 -> LDS
//   2. T_n = P(H) + Pi(H) on a halo of 2 (finite differences of u_n)
//   3. sigma_n = dt S_n / c = (dt/c)(rho0 b + Div T_n) on a halo of 1
//   4. per node: pull f(t_{n+1})_q = fc'_q(X - e_q) + dt psi_q(S_n(X - e_q));
//      at walls the modified bounce-back / anti-bounce-back rules of Sect. 3.3
//      from the node's own post-collision populations and T_n(X);
//      u_{n+1} = u_n + dt/(2 rho0) (j(t_{n+1}) + j(t_n)) with both j carrying S_n;
//      fc'_{n+1} = (1 - omega) f + omega f_eq(r, M1, M2); write fc', u.
// HBM traffic per node and step: 9 populations read and written, u read and
// written (FP64): 176 B in FP64, 104 B in FP32 storage.
#include "mclbm_internal.hpp"

namespace mclbm {

constexpr int TX = 64, TY = 16, NT = 256;
constexpr int UX = TX + 6, UY = TY + 6;    // u tile, halo 3
constexpr int TTX = TX + 4, TTY = TY + 4;  // T tile, halo 2
constexpr int SX = TX + 2, SY = TY + 2;    // sigma tile, halo 1

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of
// tiles (row-major), so that the halo rows a tile re-reads sit in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
    const int q = nblk / 8, r = nblk % 8;
    const int xcd = bid % 8, k = bid / 8;
    return xcd * q + min(xcd, r) + k;
}

// wrap an index that is at most one period out of range
__device__ __forceinline__ int wrap1(int g, int n) { return g < 0 ? g + n : (g >= n ? g - n : g); }

// ---- step ---------------------------------------------------------------------------

template <typename T, int MAT>
__global__ __launch_bounds__(NT) void step_kernel(StepArgs a) {
    const Geometry g = a.g;
    const int ntx = (g.nx + TX - 1) / TX;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int tid = threadIdx.x;
    const size_t plane = (size_t)g.ny * g.pitch;

    __shared__ double su[2][UY][UX];
    __shared__ T sT[4][TTY][TTX];
    // sigma reuses the u buffer once T is built
    T(*ss)[SY][SX] = reinterpret_cast<T(*)[SY][SX]>(&su[0][0][0]);
    static_assert(sizeof(T) * 2 * SY * SX <= sizeof(double) * 2 * UY * UX, "alias");

    const double* __restrict__ u = a.usrc;

    // 1. u_n on the tile + halo 3
    for (int i = tid; i < UX * UY; i += NT) {
        const int lx = i % UX, ly = i / UX;
        int gx = x0 - 3 + lx, gy = y0 - 3 + ly;
        if (g.px) gx = wrap(gx, g.nx);
        if (g.py) gy = wrap(gy, g.ny);
        double vx = 0.0, vy = 0.0;
        if (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny) {
            const size_t o = (size_t)gy * g.pitch + gx;
            vx = u[o];
            vy = u[plane + o];
        }
        su[0][ly][lx] = vx;
        su[1][ly][lx] = vy;
    }
    __syncthreads();

    // 2. T_n = P(H) + Pi(H) on the tile + halo 2
    for (int i = tid; i < TTX * TTY; i += NT) {
        const int lx = i % TTX, ly = i / TTX;
        int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
        if (g.px) gx = wrap(gx, g.nx);
        if (g.py) gy = wrap(gy, g.ny);
        T t[4] = {T(0), T(0), T(0), T(0)};
        if (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny) {
            const int cx = lx + 1, cy = ly + 1;  // position in su
            int xl = cx - 1, xr = cx + 1, yl = cy - 1, yr = cy + 1;
            double fx = 0.5 * a.k.inv_dx, fy = 0.5 * a.k.inv_dx;
            if (at_low(gx, g.px)) { xl = cx; fx = a.k.inv_dx; }
            else if (at_high(gx, g.nx, g.px)) { xr = cx; fx = a.k.inv_dx; }
            if (at_low(gy, g.py)) { yl = cy; fy = a.k.inv_dx; }
            else if (at_high(gy, g.ny, g.py)) { yr = cy; fy = a.k.inv_dx; }
            const double hxx = (su[0][cy][xr] - su[0][cy][xl]) * fx;
            const double hyx = (su[1][cy][xr] - su[1][cy][xl]) * fx;
            const double hxy = (su[0][yr][cx] - su[0][yl][cx]) * fy;
            const double hyy = (su[1][yr][cx] - su[1][yl][cx]) * fy;
            excess_stress<T, MAT>(T(hxx), T(hxy), T(hyx), T(hyy), T(a.k.lam), T(a.k.mu), t);
        }
        sT[0][ly][lx] = t[0];
        sT[1][ly][lx] = t[1];
        sT[2][ly][lx] = t[2];
        sT[3][ly][lx] = t[3];
    }
    __syncthreads();

    // 3. sigma_n = (dt/c) S_n on the tile + halo 1
    for (int i = tid; i < SX * SY; i += NT) {
        const int lx = i % SX, ly = i / SX;
        int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        if (g.px) gx = wrap(gx, g.nx);
        if (g.py) gy = wrap(gy, g.ny);
        T sx = T(0), sy = T(0);
        if (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny) {
            const int cx = lx + 1, cy = ly + 1;  // position in sT
            int xl = cx - 1, xr = cx + 1, yl = cy - 1, yr = cy + 1;
            T fx = T(0.5), fy = T(0.5);
            if (at_low(gx, g.px)) { xl = cx; fx = T(1); }
            else if (at_high(gx, g.nx, g.px)) { xr = cx; fx = T(1); }
            if (at_low(gy, g.py)) { yl = cy; fy = T(1); }
            else if (at_high(gy, g.ny, g.py)) { yr = cy; fy = T(1); }
            const T dxx = (sT[0][cy][xr] - sT[0][cy][xl]) * fx;
            const T dxy = (sT[1][yr][cx] - sT[1][yl][cx]) * fy;
            const T dyx = (sT[2][cy][xr] - sT[2][cy][xl]) * fx;
            const T dyy = (sT[3][yr][cx] - sT[3][yl][cx]) * fy;
            sx = T(a.k.inv_c2) * (dxx + dxy) + T(a.k.sig_b[0]);
            sy = T(a.k.inv_c2) * (dyx + dyy) + T(a.k.sig_b[1]);
        }
        ss[0][ly][lx] = sx;
        ss[1][ly][lx] = sy;
    }
    __syncthreads();

    // 4. streaming, walls, displacement update and collision per node
    const T* __restrict__ fs = reinterpret_cast<const T*>(a.fsrc);
    T* __restrict__ fd = reinterpret_cast<T*>(a.fdst);
    const int lxo = tid & 63, lyo = tid >> 6;
    const T om = T(a.k.omega);
    for (int k = 0; k < TY / 4; k++) {
        const int ly = lyo + 4 * k;
        const int gx = x0 + lxo, gy = y0 + ly;
        if (gx >= g.nx || gy >= g.ny) continue;
        const size_t o = (size_t)gy * g.pitch + gx;
        const int cx = lxo + 1, cy = ly + 1;  // position in ss
        const T sgx = ss[0][cy][cx], sgy = ss[1][cy][cx];

        T fo[9];  // own post-collision populations without forcing
#pragma unroll
        for (int q = 0; q < 9; q++) fo[q] = fs[q * plane + o];

        const bool onL = at_low(gx, g.px), onR = at_high(gx, g.nx, g.px);
        const bool onB = at_low(gy, g.py), onT = at_high(gy, g.ny, g.py);
        const bool wall = onL || onR || onB || onT;

        T f[9];
#pragma unroll
        for (int p = 0; p < 9; p++) {
            int sxp = gx - ex(p), syp = gy - ey(p);
            bool crx = false, cry = false;
            if (g.px) sxp = wrap1(sxp, g.nx); else crx = sxp < 0 || sxp >= g.nx;
            if (g.py) syp = wrap1(syp, g.ny); else cry = syp < 0 || syp >= g.ny;
            if (!crx && !cry) {
                const T gxs = ss[0][cy - ey(p)][cx - ex(p)];
                const T gys = ss[1][cy - ey(p)][cx - ex(p)];
                f[p] = fs[p * plane + (size_t)syp * g.pitch + sxp] +
                       T(3) * wq<T>(p) * (T(ex(p)) * gxs + T(ey(p)) * gys);
            } else {
                f[p] = T(0);  // set by the wall rules below
            }
        }

        if (wall) {
            // moments of the node's own populations at t_n (the collision keeps
            // r and Pi, and psi has no zeroth or second moment)
            double r = 0, mxx = 0, myy = 0;
#pragma unroll
            for (int q = 0; q < 9; q++) {
                r += (double)fo[q];
                mxx += (double)(ex(q) * ex(q)) * (double)fo[q];
                myy += (double)(ey(q) * ey(q)) * (double)fo[q];
            }
            const int tcx = lxo + 2, tcy = ly + 2;  // position in sT
            const double Txx = sT[0][tcy][tcx], Txy = sT[1][tcy][tcx];
            const double Tyx = sT[2][tcy][tcx], Tyy = sT[3][tcy][tcx];
            const int wx = onL ? SIDE_L : SIDE_R, wy = onB ? SIDE_B : SIDE_T;
            // Pi_bd / c^2 of the x wall and the y wall (Sect. 3.3): normal row and
            // column from the traction balance, tangential entry from the node
            const double sxw = onL ? -1.0 : 1.0, syw = onB ? -1.0 : 1.0;
            const double ic2 = a.k.inv_c2;
            const double Xxx = (-sxw * a.w.val[wx][0] + Txx) * ic2;
            const double Xxy = (-sxw * a.w.val[wx][1] + Tyx) * ic2;
            const double Yyy = (-syw * a.w.val[wy][1] + Tyy) * ic2;
            const double Yxy = (-syw * a.w.val[wy][0] + Txy) * ic2;
#pragma unroll
            for (int p = 1; p < 9; p++) {
                const int sxp = gx - ex(p), syp = gy - ey(p);
                const bool crx = !g.px && (sxp < 0 || sxp >= g.nx);
                const bool cry = !g.py && (syp < 0 || syp >= g.ny);
                if (!crx && !cry) continue;
                const int q = opp(p);  // the outgoing link the wall reflects
                const double fcq = (double)fo[q] + 3.0 * wq<double>(q) *
                                   ((double)ex(q) * (double)sgx + (double)ey(q) * (double)sgy);
                double jx = 0.0, jy = 0.0;
                int nd = 0;
                if (crx && a.w.bc[wx] == BC_DIR) { jx += a.w.val[wx][0]; jy += a.w.val[wx][1]; nd++; }
                if (cry && a.w.bc[wy] == BC_DIR) { jx += a.w.val[wy][0]; jy += a.w.val[wy][1]; nd++; }
                double v;
                if (nd > 0) {
                    // modified bounce-back, Eq. bbcon: -(2/cs^2) w c.j* = -6 w e.(j*/c)
                    const double s = a.k.inv_c / (double)nd;
                    v = fcq - 6.0 * wq<double>(q) * ((double)ex(q) * jx + (double)ey(q) * jy) * s;
                } else {
                    // modified anti-bounce-back, Eq. abbcon
                    double Mxx, Mxy, Myy;
                    if (crx && cry) { Mxx = Xxx; Myy = Yyy; Mxy = 0.5 * (Xxy + Yxy); }
                    else if (crx) { Mxx = Xxx; Mxy = Xxy; Myy = myy; }
                    else { Mxx = mxx; Mxy = Yxy; Myy = Yyy; }
                    const double X = ex(q), Y = ey(q);
                    const double eMe = X * X * Mxx + 2.0 * X * Y * Mxy + Y * Y * Myy;
                    const double e2 = X * X + Y * Y;
                    v = -fcq + 2.0 * wq<double>(q) *
                                   (r + 0.5 * (9.0 * eMe - 3.0 * r * e2 - 3.0 * (Mxx + Myy) + 2.0 * r));
                }
                f[p] = T(v);
            }
        }

        // moments of f(t_{n+1}) and of the own populations at t_n
        T r = T(0), m1x = T(0), m1y = T(0), m2xx = T(0), m2xy = T(0), m2yy = T(0);
        T o1x = T(0), o1y = T(0);
#pragma unroll
        for (int q = 0; q < 9; q++) {
            r += f[q];
            if (ex(q)) m1x += T(ex(q)) * f[q];
            if (ey(q)) m1y += T(ey(q)) * f[q];
            if (ex(q)) m2xx += f[q];
            if (ex(q) * ey(q)) m2xy += T(ex(q) * ey(q)) * f[q];
            if (ey(q)) m2yy += f[q];
            if (ex(q)) o1x += T(ex(q)) * fo[q];
            if (ey(q)) o1y += T(ey(q)) * fo[q];
        }

        // trapezoidal rule (Sect. 3.2): u += dt/(2 rho0) (j(t_{n+1}) + j(t_n)),
        // j(t_{n+1}) + j(t_n) = c (M1 + M1' + sigma_n)
        const double unx = u[o] + a.k.ucoef * (double)(m1x + o1x + sgx);
        const double uny = u[plane + o] + a.k.ucoef * (double)(m1y + o1y + sgy);
        a.udst[o] = unx;
        a.udst[plane + o] = uny;

        // BGK collision without the forcing term
#pragma unroll
        for (int q = 0; q < 9; q++) {
            const T e = feq_q<T>(q, r, m1x, m1y, m2xx, m2xy, m2yy);
            fd[q * plane + o] = f[q] + om * (e - f[q]);
        }
    }
}

// ---- step, y-marching form ------------------------------------------------------------------
//
// The same step without LDS or barriers.  Each wave owns a strip of MO = 58
// columns (lanes 3..60, halo lanes 0..2 and 61..63) and marches down a chunk of
// rows.  At iteration r it holds in registers the rows r..r+3 of u, r..r+2 of
// T, r-1..r+1 of sigma and r-1..r+1 of the populations; x neighbours come from
// lane shuffles, y neighbours from the rows it holds.  Every population and u
// value of the strip is loaded once (the next rows one iteration ahead), plus
// the halo columns and the rows that prime the pipeline of a chunk.

constexpr int MH = 3, MO = 64 - 2 * MH;

template <typename V>
__device__ __forceinline__ V from_prev(V v) { return __shfl_up(v, 1); }    // value of lane l-1
template <typename V>
__device__ __forceinline__ V from_next(V v) { return __shfl_down(v, 1); }  // value of lane l+1

template <typename T, int MAT>
__global__ __launch_bounds__(256) void march_kernel(StepArgs a, int nstrip, int nchunk, int chunk) {
    const Geometry g = a.g;
    const int lane = threadIdx.x & 63;
    const int item = xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (item >= nstrip * nchunk) return;  // uniform per wave
    const int strip = item % nstrip, chk = item / nstrip;
    const int gxu = strip * MO - MH + lane;  // unwrapped column of this lane
    int x = gxu;
    bool xin;
    if (g.px) { x = wrap(gxu, g.nx); xin = true; }
    else xin = gxu >= 0 && gxu < g.nx;
    const bool own = lane >= MH && lane < MH + MO && gxu < g.nx;
    const bool pop = xin && lane >= MH - 1 && lane <= MH + MO;  // lanes whose populations are pulled
    const bool atL = xin && at_low(x, g.px), atR = xin && at_high(x, g.nx, g.px);
    const int yc = chk * chunk, ye = min(yc + chunk, g.ny);
    const size_t plane = (size_t)g.ny * g.pitch;
    const T* __restrict__ fs = reinterpret_cast<const T*>(a.fsrc);
    T* __restrict__ fd = reinterpret_cast<T*>(a.fdst);
    const double* __restrict__ u = a.usrc;
    const double idx = a.k.inv_dx;
    const T ic2 = T(a.k.inv_c2), sbx = T(a.k.sig_b[0]), sby = T(a.k.sig_b[1]);
    const T lam = T(a.k.lam), mu = T(a.k.mu);

    auto row_of = [&](int r, int& rr) -> bool {
        if (g.py) { rr = wrap(r, g.ny); return true; }
        rr = r;
        return r >= 0 && r < g.ny;
    };
    auto load_u = [&](int r, double v[2]) {
        int rr;
        v[0] = 0.0; v[1] = 0.0;
        if (xin && row_of(r, rr)) {
            const size_t o = (size_t)rr * g.pitch + x;
            v[0] = u[o];
            v[1] = u[plane + o];
        }
    };
    auto load_f = [&](int r, T f[9]) {
        int rr;
        if (pop && row_of(r, rr)) {
            const size_t o = (size_t)rr * g.pitch + x;
#pragma unroll
            for (int q = 0; q < 9; q++) f[q] = fs[q * plane + o];
        } else {
#pragma unroll
            for (int q = 0; q < 9; q++) f[q] = T(0);
        }
    };
    // T = P(H) + Pi(H) at row r from u at rows r-1, r, r+1 of this lane
    auto stress = [&](int r, const double um[2], const double u0[2], const double up[2], T t[4]) {
        const double lx = from_prev(u0[0]), rx = from_next(u0[0]);
        const double ly = from_prev(u0[1]), ry = from_next(u0[1]);
        t[0] = t[1] = t[2] = t[3] = T(0);
        int rr;
        if (!(xin && row_of(r, rr))) return;
        double ax = lx, bx = rx, ay = ly, by = ry, fx = 0.5 * idx;
        if (atL) { ax = u0[0]; ay = u0[1]; fx = idx; }
        else if (atR) { bx = u0[0]; by = u0[1]; fx = idx; }
        double cx = um[0], dx = up[0], cy = um[1], dy = up[1], fy = 0.5 * idx;
        if (!g.py && rr == 0) { cx = u0[0]; cy = u0[1]; fy = idx; }
        else if (!g.py && rr == g.ny - 1) { dx = u0[0]; dy = u0[1]; fy = idx; }
        excess_stress<T, MAT>(T((bx - ax) * fx), T((dx - cx) * fy), T((by - ay) * fx), T((dy - cy) * fy),
                              lam, mu, t);
    };
    // sigma = dt S / c at row r from T at rows r-1, r, r+1 of this lane
    auto sigma = [&](int r, const T tm[4], const T t0[4], const T tp[4], T sg[2]) {
        const T lxx = from_prev(t0[0]), rxx = from_next(t0[0]);
        const T lyx = from_prev(t0[2]), ryx = from_next(t0[2]);
        sg[0] = sg[1] = T(0);
        int rr;
        if (!(xin && row_of(r, rr))) return;
        T axx = lxx, bxx = rxx, ayx = lyx, byx = ryx, fx = T(0.5);
        if (atL) { axx = t0[0]; ayx = t0[2]; fx = T(1); }
        else if (atR) { bxx = t0[0]; byx = t0[2]; fx = T(1); }
        T cxy = tm[1], dxy = tp[1], cyy = tm[3], dyy = tp[3], fy = T(0.5);
        if (!g.py && rr == 0) { cxy = t0[1]; cyy = t0[3]; fy = T(1); }
        else if (!g.py && rr == g.ny - 1) { dxy = t0[1]; dyy = t0[3]; fy = T(1); }
        sg[0] = ic2 * ((bxx - axx) * fx + (dxy - cxy) * fy) + sbx;
        sg[1] = ic2 * ((byx - ayx) * fx + (dyy - cyy) * fy) + sby;
    };

    // prime the pipeline for the first iteration r = yc - 2
    double U0[2], U1[2], U2[2], U3[2], Un[2], tmp[2];
    T T0[4], T1[4], T2[4];
    T Gm[2] = {T(0), T(0)}, G0[2] = {T(0), T(0)}, G1[2];
    T Fm[9], F0[9], F1[9], Fn[9];
    load_u(yc - 3, tmp);
    load_u(yc - 2, U0);
    load_u(yc - 1, U1);
    load_u(yc, U2);
    load_u(yc + 1, Un);
    load_f(yc - 1, Fn);
    stress(yc - 2, tmp, U0, U1, T0);
    stress(yc - 1, U0, U1, U2, T1);
#pragma unroll
    for (int q = 0; q < 9; q++) { Fm[q] = T(0); F0[q] = T(0); }

    for (int r = yc - 2; r < ye; r++) {
        U3[0] = Un[0]; U3[1] = Un[1];
#pragma unroll
        for (int q = 0; q < 9; q++) F1[q] = Fn[q];
        if (r + 1 < ye) {  // next rows, one iteration ahead
            load_u(r + 4, Un);
            load_f(r + 2, Fn);
        }
        stress(r + 2, U1, U2, U3, T2);
        sigma(r + 1, T0, T1, T2, G1);

        if (r >= yc) {
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

            const bool onB = at_low(r, g.py), onT = at_high(r, g.ny, g.py);
            if (own && (atL || atR || onB || onT)) {
                double rr0 = 0, mxx = 0, myy = 0;
#pragma unroll
                for (int q = 0; q < 9; q++) {
                    rr0 += (double)F0[q];
                    mxx += (double)(ex(q) * ex(q)) * (double)F0[q];
                    myy += (double)(ey(q) * ey(q)) * (double)F0[q];
                }
                const double Txx = T0[0], Txy = T0[1], Tyx = T0[2], Tyy = T0[3];
                const int wx = atL ? SIDE_L : SIDE_R, wy = onB ? SIDE_B : SIDE_T;
                const double sxw = atL ? -1.0 : 1.0, syw = onB ? -1.0 : 1.0;
                const double c2i = a.k.inv_c2;
                const double Xxx = (-sxw * a.w.val[wx][0] + Txx) * c2i;
                const double Xxy = (-sxw * a.w.val[wx][1] + Tyx) * c2i;
                const double Yyy = (-syw * a.w.val[wy][1] + Tyy) * c2i;
                const double Yxy = (-syw * a.w.val[wy][0] + Txy) * c2i;
#pragma unroll
                for (int p = 1; p < 9; p++) {
                    const bool crx = (ex(p) > 0 && atL) || (ex(p) < 0 && atR);
                    const bool cry = (ey(p) > 0 && onB) || (ey(p) < 0 && onT);
                    if (!crx && !cry) continue;
                    const int q = opp(p);  // the outgoing link the wall reflects
                    const double fcq = (double)F0[q] + 3.0 * wq<double>(q) *
                                       ((double)ex(q) * (double)G0[0] + (double)ey(q) * (double)G0[1]);
                    double jx = 0.0, jy = 0.0;
                    int nd = 0;
                    if (crx && a.w.bc[wx] == BC_DIR) { jx += a.w.val[wx][0]; jy += a.w.val[wx][1]; nd++; }
                    if (cry && a.w.bc[wy] == BC_DIR) { jx += a.w.val[wy][0]; jy += a.w.val[wy][1]; nd++; }
                    double v;
                    if (nd > 0) {
                        // modified bounce-back, Eq. bbcon
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
                        v = -fcq + 2.0 * wq<double>(q) *
                                       (rr0 + 0.5 * (9.0 * eMe - 3.0 * rr0 * e2 - 3.0 * (Mxx + Myy) + 2.0 * rr0));
                    }
                    f[p] = T(v);
                }
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
            if (own) {
                const size_t o = (size_t)r * g.pitch + x;
                a.udst[o] = U0[0] + a.k.ucoef * (double)(m1x + o1x + G0[0]);
                a.udst[plane + o] = U0[1] + a.k.ucoef * (double)(m1y + o1y + G0[1]);
                const T om = T(a.k.omega);
#pragma unroll
                for (int q = 0; q < 9; q++) {
                    const T e = feq_q<T>(q, rho, m1x, m1y, m2xx, m2xy, m2yy);
                    fd[q * plane + o] = f[q] + om * (e - f[q]);
                }
            }
        }
        // rotate the rows
        U0[0] = U1[0]; U0[1] = U1[1];
        U1[0] = U2[0]; U1[1] = U2[1];
        U2[0] = U3[0]; U2[1] = U3[1];
#pragma unroll
        for (int c = 0; c < 4; c++) { T0[c] = T1[c]; T1[c] = T2[c]; }
        Gm[0] = G0[0]; Gm[1] = G0[1];
        G0[0] = G1[0]; G0[1] = G1[1];
#pragma unroll
        for (int q = 0; q < 9; q++) { Fm[q] = F0[q]; F0[q] = F1[q]; }
    }
}

// ---- per-node helpers for init, read-out and diagnostics (FP64, global loads) ----------

__device__ __forceinline__ double ld_u(const InitLike& a, int c, int gx, int gy) {
    return a.u[(size_t)c * a.g.ny * a.g.pitch + (size_t)gy * a.g.pitch + gx];
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
    const size_t plane = (size_t)a.b.g.ny * a.b.g.pitch;
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
    const size_t plane = (size_t)g.ny * g.pitch;
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
        const size_t plane = (size_t)g.ny * g.pitch;
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

template <typename T>
static hipError_t step_t(int material, const StepArgs& a, hipStream_t st) {
    const int nstrip = (a.g.nx + MO - 1) / MO;
    const int chunk = march_chunk(a.g, nstrip);
    const int nchunk = (a.g.ny + chunk - 1) / chunk;
    const dim3 grid((nstrip * nchunk + 3) / 4), block(256);
    switch (material) {
    case MAT_SVK: hipLaunchKernelGGL((march_kernel<T, MAT_SVK>), grid, block, 0, st, a, nstrip, nchunk, chunk); break;
    case MAT_NH: hipLaunchKernelGGL((march_kernel<T, MAT_NH>), grid, block, 0, st, a, nstrip, nchunk, chunk); break;
    default: hipLaunchKernelGGL((march_kernel<T, MAT_LIN>), grid, block, 0, st, a, nstrip, nchunk, chunk); break;
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
