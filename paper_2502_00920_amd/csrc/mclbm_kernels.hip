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

template <typename T>
static hipError_t step_t(int material, const StepArgs& a, hipStream_t st) {
    const int ntx = (a.g.nx + TX - 1) / TX, nty = (a.g.ny + TY - 1) / TY;
    const dim3 grid(ntx * nty), block(NT);
    switch (material) {
    case MAT_SVK: hipLaunchKernelGGL((step_kernel<T, MAT_SVK>), grid, block, 0, st, a); break;
    case MAT_NH: hipLaunchKernelGGL((step_kernel<T, MAT_NH>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((step_kernel<T, MAT_LIN>), grid, block, 0, st, a); break;
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
