// Device-side building blocks of the moment-chain LBM step (gfx950).
//
// Everything on the device works in lattice-scaled moments of the populations:
//   r = sum f,  M1 = sum e f,  M2 = sum e e f
// with e_q the integer D2Q9 directions (Tab. 1), so that the physical moments
// are j = c M1 and Pi = c^2 M2 (c = dX/dt = sqrt(3) c_s, Sect. 3.2).  In these
// variables the equilibrium of Sect. 3.2 is free of c:
//   f_eq,q = w_q [ r + 3 e.M1 + (9 e.M2.e - 3 r |e|^2 - 3 tr M2 + 2 r) / 2 ]
// the forcing term of Eq. forcing scaled by dt is dt psi_q = 3 w_q e.sigma with
// sigma = dt S / c, the Dirichlet correction of Eq. bbcon is
// -6 w_q e.(j*/c), and the Neumann rule of Eq. abbcon uses the same
// expression as f_eq with M2 = Pi_bd / c^2 and no M1 term.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mclbm {

// ---- kernel arguments ---------------------------------------------------------

struct Geometry {
    int nx, ny;        // nodes
    int pitch;         // row pitch in elements (multiple of 64)
    int px, py;        // periodic in x / y
    long long plane;   // elements per component: ny rows of pitch
};

// The state (u and the populations) is stored in row records: lattice row y
// keeps the rows of all its components side by side, [ny][component][pitch],
// so that a wave's loads and stores of one lattice row fall in one stretch of
// memory.  (On the 8192^2 lattice the step's access pattern alone ran 8-16 %
// faster so than with one plane per component, [component][ny][pitch].)
//   u (and the j0 of init): [ny][2][pitch] doubles;
//   populations, FP64 / FP32: [ny][9][pitch];
//   16-bit: per lattice row four rows of pitch 32-bit words (word w holds
//   population 2w in its low half, 2w + 1 in its high half), then one row of
//   pitch 16-bit values (population 8): 18 pitch bytes.
// Element index of component c of node (x, y) in a [ny][2][pitch] field:
__host__ __device__ __forceinline__ size_t u_at(const Geometry& g, int c, int y, int x) {
    return ((size_t)y * 2 + c) * (size_t)g.pitch + x;
}

struct Coef {
    double omega;     // dt / tau, tau in units of dt
    double omega_p;   // rate of the even non-equilibrium part (omega: BGK)
    double c;         // lattice speed dX/dt
    double inv_c;     // 1/c
    double inv_c2;    // 1/c^2 = dt^2/dX^2 = rho0/(3 mu)
    double inv_dx;    // 1/dX
    double ucoef;     // dX / (2 rho0): trapezoidal rule in scaled moments
    double sig_b[2];  // rho0 b dX / c^2: body-force part of sigma
    double s_from_sig;// c / dt: S = sigma * c / dt
    double lam, mu, rho0;
    double fscale;    // stored = population * fscale (a power of two; 1 except FP16 storage)
    double finv;      // 1 / fscale
    int extrap;       // Neumann wall values: 0 the node's (zeroth order), 1 linear to the wall
    int corner;       // shear entry of Pi_bd across two Neumann walls: 0 mean, 1 x wall's, 2 y wall's
};

// Wall data of one step: type per side and its value at t_n (j* for
// Dirichlet, T* for Neumann, physical units).
struct Walls {
    int bc[4];
    double val[4][2];
};

enum { SIDE_L = 0, SIDE_R = 1, SIDE_B = 2, SIDE_T = 3 };
enum { BC_DIR = 0, BC_NEU = 1, BC_PER = 2 };
enum { MAT_SVK = 0, MAT_NH = 1, MAT_LIN = 2 };
// population storage: FP64, FP32, FP16 (scaled) or BF16; arithmetic is FP64 for
// the first and FP32 for the others, the displacement FP64 always
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_F16 = 2, PREC_BF16 = 3 };

// ---- D2Q9, Tab. 1 ---------------------------------------------------------------

__host__ __device__ constexpr int ex(int q) {
    return (q == 1 || q == 5 || q == 8) ? 1 : ((q == 3 || q == 6 || q == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey(int q) {
    return (q == 2 || q == 5 || q == 6) ? 1 : ((q == 4 || q == 7 || q == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int q) {
    return q == 0 ? 0 : (q <= 4 ? ((q + 1) % 4) + 1 : ((q - 3) % 4) + 5);
}
template <typename T>
__host__ __device__ constexpr T wq(int q) {
    return q == 0 ? T(4) / T(9) : (q <= 4 ? T(1) / T(9) : T(1) / T(36));
}

// Equilibrium in scaled moments (see the file comment).
template <typename T>
__device__ __forceinline__ T feq_q(int q, T r, T m1x, T m1y, T m2xx, T m2xy, T m2yy) {
    const T X = T(ex(q)), Y = T(ey(q));
    const T eM1 = X * m1x + Y * m1y;
    const T eM2e = X * X * m2xx + T(2) * X * Y * m2xy + Y * Y * m2yy;
    const T e2 = X * X + Y * Y;
    return wq<T>(q) * (r + T(3) * eM1 +
                       T(0.5) * (T(9) * eM2e - T(3) * r * e2 - T(3) * (m2xx + m2yy) + T(2) * r));
}

// The collision of one node in FP64, written per direction pair q, qbar.  The
// non-equilibrium part n = f - feq relaxes with two rates: its odd part
// (n_q - n_qbar)/2 at omega (the paper's BGK rate) and its even part at
// omega_p (omega_p = omega is BGK; other values are the two-relaxation-time
// option).  With feq_q = w_q X_q, A = (omega_p + omega)/2, B = (omega_p - omega)/2:
//   fn_q = (1 - A) f_q - B f_qbar + w_q (omega_p E_q + omega O_q),
// where E and O are the parts of X even and odd under q -> qbar.  The terms a
// direction shares with its opposite are formed once, the moments share the sums
// over the diagonal pairs, and the weights fold into the rates.  The result
// equals the relaxation towards feq_q above up to the rounding order.
struct CollideRates {
    double oa;         // 1 - A
    double b;          // B (0 for BGK)
    double ep0, ep1, ep5;  // omega_p w_q
    double od1, od5;   // 3 omega w_q
    double o0;         // 1 - omega_p
};
__host__ __device__ inline CollideRates collide_rates(double omega, double omega_p) {
    CollideRates k;
    k.oa = 1.0 - 0.5 * (omega_p + omega);
    k.b = 0.5 * (omega_p - omega);
    k.ep0 = omega_p * (4.0 / 9.0);
    k.ep1 = omega_p * (1.0 / 9.0);
    k.ep5 = omega_p * (1.0 / 36.0);
    k.od1 = 3.0 * omega * (1.0 / 9.0);
    k.od5 = 3.0 * omega * (1.0 / 36.0);
    k.o0 = 1.0 - omega_p;
    return k;
}
struct NodeMoments {
    double r, m1x, m1y;
};
template <bool TWO_RATES>
__device__ __forceinline__ NodeMoments collide_node(const double F[9], const CollideRates& k, double fn[9]) {
    const double a57 = F[5] + F[7], a68 = F[6] + F[8];
    const double c57 = F[5] - F[7], c86 = F[8] - F[6];
    const double s24 = F[2] + F[4], dsum = a57 + a68;
    const double m2xx = (F[1] + F[3]) + dsum, m2yy = s24 + dsum, m2xy = a57 - a68;
    const double m1x = (F[1] - F[3]) + (c57 + c86);
    const double m1y = (F[2] - F[4]) + (c57 - c86);
    const double r = F[0] + (m2xx + s24);
    const double S = m2xx + m2yy;
    const double X0 = 2.0 * r - 1.5 * S;        // rest
    const double b1 = 0.5 * r - 1.5 * S;        // axis directions, before their own terms
    const double Px = b1 + 4.5 * m2xx, Py = b1 + 4.5 * m2yy;
    const double Dg = 3.0 * S - r;              // diagonal directions
    const double Dp = Dg + 9.0 * m2xy, Dm = Dg - 9.0 * m2xy;
    const double ppl = m1x + m1y, pmi = m1x - m1y;
    const double Ex = k.ep1 * Px, Ox = k.od1 * m1x, Ey = k.ep1 * Py, Oy = k.od1 * m1y;
    const double Ep = k.ep5 * Dp, Op = k.od5 * ppl, Em = k.ep5 * Dm, Om = k.od5 * pmi;
    fn[0] = k.o0 * F[0] + k.ep0 * X0;
    fn[1] = k.oa * F[1] + (Ex + Ox);
    fn[3] = k.oa * F[3] + (Ex - Ox);
    fn[2] = k.oa * F[2] + (Ey + Oy);
    fn[4] = k.oa * F[4] + (Ey - Oy);
    fn[5] = k.oa * F[5] + (Ep + Op);
    fn[7] = k.oa * F[7] + (Ep - Op);
    fn[6] = k.oa * F[6] + (Em - Om);
    fn[8] = k.oa * F[8] + (Em + Om);
    if constexpr (TWO_RATES) {  // the even part's rate differs from omega
        fn[1] -= k.b * F[3];
        fn[3] -= k.b * F[1];
        fn[2] -= k.b * F[4];
        fn[4] -= k.b * F[2];
        fn[5] -= k.b * F[7];
        fn[7] -= k.b * F[5];
        fn[6] -= k.b * F[8];
        fn[8] -= k.b * F[6];
    }
    return NodeMoments{r, m1x, m1y};
}

// ---- materials, Sect. 4 (plane strain) ------------------------------------------------

// First Piola-Kirchhoff stress P(H), H_ab = d u_a / d X_b, order (xx, xy, yx, yy).
template <typename T, int MAT>
__device__ __forceinline__ void first_pk(T hxx, T hxy, T hyx, T hyy, T lam, T mu, T P[4]) {
    if constexpr (MAT == MAT_SVK) {
        // S = lam tr(E) I + 2 mu E, E = (H + H^T + H^T H)/2, P = (I + H) S
        const T Exx = hxx + T(0.5) * (hxx * hxx + hyx * hyx);
        const T Eyy = hyy + T(0.5) * (hxy * hxy + hyy * hyy);
        const T Exy = T(0.5) * (hxy + hyx + hxx * hxy + hyx * hyy);
        const T trE = Exx + Eyy;
        const T Sxx = lam * trE + T(2) * mu * Exx;
        const T Syy = lam * trE + T(2) * mu * Eyy;
        const T Sxy = T(2) * mu * Exy;
        P[0] = (T(1) + hxx) * Sxx + hxy * Sxy;
        P[1] = (T(1) + hxx) * Sxy + hxy * Syy;
        P[2] = hyx * Sxx + (T(1) + hyy) * Sxy;
        P[3] = hyx * Sxy + (T(1) + hyy) * Syy;
    } else if constexpr (MAT == MAT_NH) {
        // S = lam/2 (J^2 - 1) C^-1 + mu (I - C^-1), P = F S
        //   = mu (F - F^-T) + lam/2 (J^2 - 1) F^-T,   F^-T = (I + K) / J,
        // K = cof(H) = [[hyy, -hyx], [-hxy, hxx]], and with d = J - 1 = tr H + det H
        //   F - F^-T = (d I + J H - K) / J,  J^2 - 1 = d (d + 2):
        // every term is O(H), so small strains keep their relative precision.
        const T d = (hxx + hyy) + (hxx * hyy - hxy * hyx);
        const T J = T(1) + d;
        const T iJ = T(1) / J;
        const T a = T(0.5) * lam * d * (d + T(2));
        P[0] = iJ * (mu * (d + J * hxx - hyy) + a * (T(1) + hyy));
        P[1] = iJ * (mu * (J * hxy + hyx) - a * hyx);
        P[2] = iJ * (mu * (J * hyx + hxy) - a * hxy);
        P[3] = iJ * (mu * (d + J * hyy - hxx) + a * (T(1) + hxx));
    } else {
        // Hooke's law of the linear-elastic scheme
        const T tr = hxx + hyy;
        P[0] = lam * tr + mu * (hxx + hxx);
        P[1] = mu * (hxy + hyx);
        P[2] = mu * (hyx + hxy);
        P[3] = lam * tr + mu * (hyy + hyy);
    }
}

// T = P(H) + Pi(H) with the stress of the bare chain Pi(H) = -mu (H + H^T + tr H I)
// (Sect. 3.1: the source carries the divergence of T).
template <typename T, int MAT>
__device__ __forceinline__ void excess_stress(T hxx, T hxy, T hyx, T hyy, T lam, T mu, T out[4]) {
    if constexpr (MAT == MAT_LIN) {
        // P_lin + Pi(H) = (lam - mu) tr H I: exactly zero at nu = 1/4
        const T d = (lam - mu) * (hxx + hyy);
        out[0] = d; out[1] = T(0); out[2] = T(0); out[3] = d;
    } else {
        T P[4];
        first_pk<T, MAT>(hxx, hxy, hyx, hyy, lam, mu, P);
        const T tr = hxx + hyy;
        const T sh = mu * (hxy + hyx);
        out[0] = P[0] - mu * (hxx + hxx + tr);
        out[1] = P[1] - sh;
        out[2] = P[2] - sh;
        out[3] = P[3] - mu * (hyy + hyy + tr);
    }
}

// ---- finite differences, Sect. 3.2 ----------------------------------------------------
// Central differences in the interior, first-order one-sided differences with the
// inward neighbour at the outermost node of a non-periodic axis.

__device__ __forceinline__ bool at_low(int g, int per) { return !per && g == 0; }
__device__ __forceinline__ bool at_high(int g, int n, int per) { return !per && g == n - 1; }

__device__ __forceinline__ int wrap(int g, int n) {
    int r = g % n;
    return r < 0 ? r + n : r;
}

}  // namespace mclbm
