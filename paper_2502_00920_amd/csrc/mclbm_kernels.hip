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
//   5. fc'_{n+1} = f - omega odd(f - f_eq) - omega_p even(f - f_eq), f_eq =
//      f_eq(r, M1, M2): BGK for omega_p = omega (the paper's), two relaxation
//      times otherwise
// A step is one launch of march_kernel: one pass over HBM, each wave owning 64
// aligned columns of a band of rows; the waves that touch a lattice edge apply
// the wall rules to their wall nodes.
// HBM traffic per node and step: 9 populations read and written, u read and
// written (FP64): 176 B in FP64, 104 B in FP32 storage.
#include <algorithm>
#include <mutex>
#include <type_traits>

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
// wave-uniform SGPR offset and a 32-bit byte offset per lane.  The march takes
// one resource per displacement buffer and, for the populations, one per lattice
// row (its record), so that no 32-bit range limits the population buffers.
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
// Streaming stores (nt): the new state is read back only in the next step, long
// after it has left the caches, so it should not displace the lines that the
// halo reads of neighbouring strips reuse.
constexpr int kCpolNT = 2;
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t r, uint32_t ob, uint32_t so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, ob, so, kCpolNT);
}
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t r, uint32_t ob, uint32_t so, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, ob, so, kCpolNT);
}

// ---- population storage formats ----------------------------------------------------------
//
// FP64 and FP32: nine rows of double / float per lattice row.  FP16 and BF16: the
// populations two per 32-bit word in four rows (word w holds population 2w in its
// low half and 2w + 1 in its high half) and population 8 in a fifth row of 16-bit
// values, 18 bytes per node.  In this scheme the rest state has f = 0, so the stored values
// are the deviation from that equilibrium.  FP16 values are the populations times a
// power of two (Coef::fscale) that keeps them out of the subnormal range; BF16 has
// FP32's exponent range and is stored unscaled.  Arithmetic is FP32 for all three.

__device__ __forceinline__ uint32_t f16_bits(float v) {
    return __builtin_bit_cast(unsigned short, (_Float16)v);  // round to nearest even
}
__device__ __forceinline__ float f16_value(uint32_t b) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(b & 0xffffu));
}
__device__ __forceinline__ uint32_t bf16_bits(float v) {
    return __builtin_bit_cast(unsigned short, (__bf16)v);  // round to nearest even (v_cvt_pk_bf16_f32)
}
__device__ __forceinline__ float bf16_value(uint32_t b) { return __builtin_bit_cast(float, (b & 0xffffu) << 16); }

template <int PR>
struct Store {  // PREC_F64, PREC_F32: plain values
    using T = typename std::conditional<PR == PREC_F64, double, float>::type;  // arithmetic
    using TS = T;  // stresses, source and their halo
    using ST = T;  // storage
    static constexpr bool packed = false;
};
template <>
struct Store<PREC_F16> {
    using T = float;
    using TS = float;
    using ST = uint16_t;
    static constexpr bool packed = true;
    __device__ static uint32_t enc(float v) { return f16_bits(v); }
    __device__ static float dec(uint32_t b) { return f16_value(b); }
};
template <>
struct Store<PREC_BF16> {
    using T = float;
    using TS = float;
    using ST = uint16_t;
    static constexpr bool packed = true;
    __device__ static uint32_t enc(float v) { return bf16_bits(v); }
    __device__ static float dec(uint32_t b) { return bf16_value(b); }
};

// bytes of one lattice row's record of populations (see u_at for the layout)
template <int PR>
__host__ __device__ constexpr uint32_t pop_row_bytes(int pitch) {
    return (uint32_t)pitch * (PR == PREC_F64 ? 72u : (PR == PREC_F32 ? 36u : 18u));
}

// population q of node (x, y), for the per-node kernels
template <int PR>
__device__ __forceinline__ double pop_get(const void* f, const Geometry& g, int y, int x, int q, double finv) {
    using S = Store<PR>;
    if constexpr (!S::packed) {
        return (double)reinterpret_cast<const typename S::ST*>(f)[((size_t)y * 9 + q) * g.pitch + x];
    } else {
        const size_t row = (size_t)y * 9 * g.pitch;  // the record's first 16-bit unit
        if (q == 8) return (double)S::dec(reinterpret_cast<const uint16_t*>(f)[row + 8 * (size_t)g.pitch + x]) * finv;
        const uint32_t v = reinterpret_cast<const uint32_t*>(f)[row / 2 + (size_t)(q >> 1) * g.pitch + x];
        return (double)S::dec((q & 1) ? (v >> 16) : v) * finv;
    }
}
template <int PR>
__device__ __forceinline__ void pop_put_all(void* f, const Geometry& g, int y, int x, const double v[9], double fscale) {
    using S = Store<PR>;
    if constexpr (!S::packed) {
        for (int q = 0; q < 9; q++)
            reinterpret_cast<typename S::ST*>(f)[((size_t)y * 9 + q) * g.pitch + x] = (typename S::ST)v[q];
    } else {
        const size_t row = (size_t)y * 9 * g.pitch;
        uint32_t* w = reinterpret_cast<uint32_t*>(f);
        for (int k = 0; k < 4; k++)
            w[row / 2 + (size_t)k * g.pitch + x] =
                S::enc((float)(v[2 * k] * fscale)) | (S::enc((float)(v[2 * k + 1] * fscale)) << 16);
        reinterpret_cast<uint16_t*>(f)[row + 8 * (size_t)g.pitch + x] = (uint16_t)S::enc((float)(v[8] * fscale));
    }
}

// ---- lane shifts across the wave (DPP wave_shr:1 / wave_shl:1, one VALU move per dword)

constexpr int kDppWaveShr1 = 0x138;  // lane l reads lane l-1
constexpr int kDppWaveShl1 = 0x130;  // lane l reads lane l+1

template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v, double edge) {
    const u32x2 a = __builtin_bit_cast(u32x2, v), e = __builtin_bit_cast(u32x2, edge);
    u32x2 r;
    r.x = (unsigned)__builtin_amdgcn_update_dpp((int)e.x, (int)a.x, CTRL, 0xf, 0xf, false);
    r.y = (unsigned)__builtin_amdgcn_update_dpp((int)e.y, (int)a.y, CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, r);
}
// value of lane l-1; lane 0 gets edge
template <typename V>
__device__ __forceinline__ V from_prev(V v, V edge) { return dpp_shift<kDppWaveShr1>(v, edge); }
// value of lane l+1; lane 63 gets edge
template <typename V>
__device__ __forceinline__ V from_next(V v, V edge) { return dpp_shift<kDppWaveShl1>(v, edge); }

// ---- wall rules (Sect. 3.3), FP64 ----------------------------------------------------------
//
// The links of a wall node whose source lies beyond a wall, in FP64 in every
// storage mode (the boundary-traction balance: T* and P(H) N nearly cancel on a
// loaded wall), from the node's own post-collision populations fo (without the
// forcing), its sigma (g0x, g0y) and its stresses td = P(H) + Pi(H) at t_n:
// modified bounce-back (Eq. bbcon) across Dirichlet sides; modified
// anti-bounce-back (Eq. abbcon) across Neumann sides, with Pi_bd N =
// -T* + (P + Pi(H)) N in the wall's normal row and column and the population
// moment Pi in the tangential entry, carried to the half-way wall at zeroth order
// or, with k.extrap, linearly from the inward node (txx_i, tyx_i, myi: T_xx, T_yx
// and the population Pi_yy / c^2 of the x wall's inward node; txy_i, tyy_i, mxi:
// T_xy, T_yy and Pi_xx / c^2 of the y wall's).  A link crossing a Dirichlet and a Neumann
// side takes the Dirichlet rule, one crossing two Dirichlet sides the mean of
// their j*, one crossing two Neumann sides the Pi_bd with both normal rows from
// the tractions and the shear entry by k.corner (the mean of the two walls' by
// default).  atL / atR: the node is on the left / right wall (non-periodic x);
// wyB / wyT: on the bottom / top wall.  Writes the incoming populations into fd.
template <typename F>
__device__ __forceinline__ void apply_walls(const Walls& W, const Coef& k, bool atL, bool atR, bool wyB, bool wyT,
                                            const F fo[9], double g0x, double g0y, const double td[4],
                                            double txx_i, double tyx_i, double myi, double txy_i, double tyy_i,
                                            double mxi, double fd[9]) {
    const double ic2 = k.inv_c2, icd = k.inv_c;
    // r and the second moments: the collision keeps them and psi has neither
    const double d5 = (double)fo[5] + (double)fo[7], d6 = (double)fo[6] + (double)fo[8];
    const double a13 = (double)fo[1] + (double)fo[3], a24 = (double)fo[2] + (double)fo[4];
    const double r0 = (double)fo[0] + a13 + a24 + (d5 + d6);
    const double mxx = a13 + (d5 + d6);
    const double myy = a24 + (d5 + d6);
    const bool lin = k.extrap != 0;
    auto ext = [&](double v, double vin) { return lin ? 0.5 * (3.0 * v - vin) : v; };
    const bool wx = atL || atR, wy = wyB || wyT;
    const int sx = atL ? SIDE_L : SIDE_R, sy = wyB ? SIDE_B : SIDE_T;
    const double nxo = atL ? -1.0 : 1.0, nyo = wyB ? -1.0 : 1.0;  // outward normals
    // Pi_bd / c^2 of each Neumann wall, (xx, xy, yy)
    double PX[3] = {0.0, 0.0, 0.0}, PY[3] = {0.0, 0.0, 0.0};
    if (wx && W.bc[sx] == BC_NEU) {
        PX[0] = (-nxo * W.val[sx][0] + ext(td[0], txx_i)) * ic2;
        PX[1] = (-nxo * W.val[sx][1] + ext(td[2], tyx_i)) * ic2;
        PX[2] = ext(myy, myi);
    }
    if (wy && W.bc[sy] == BC_NEU) {
        PY[0] = ext(mxx, mxi);
        PY[1] = (-nyo * W.val[sy][0] + ext(td[1], txy_i)) * ic2;
        PY[2] = (-nyo * W.val[sy][1] + ext(td[3], tyy_i)) * ic2;
    }
    const double PCxy = k.corner == 1 ? PX[1] : (k.corner == 2 ? PY[1] : 0.5 * (PX[1] + PY[1]));
#pragma unroll
    for (int q = 1; q < 9; q++) {
        const int X = ex(q), Y = ey(q);
        const bool cx = (atL && X < 0) || (atR && X > 0);  // the link leaves across the x wall
        const bool cy = (wyB && Y < 0) || (wyT && Y > 0);  // ... across the y wall
        if (!cx && !cy) continue;
        const double w = wq<double>(q);
        const double fcq = (double)fo[q] + 3.0 * w * (X * g0x + Y * g0y);  // post-collision with forcing
        const bool dx_ = cx && W.bc[sx] == BC_DIR, dy_ = cy && W.bc[sy] == BC_DIR;
        double val;
        if (dx_ || dy_) {
            double jx = 0.0, jy = 0.0;
            if (dx_) { jx += W.val[sx][0] * icd; jy += W.val[sx][1] * icd; }
            if (dy_) { jx += W.val[sy][0] * icd; jy += W.val[sy][1] * icd; }
            const double kk = (dx_ && dy_) ? 0.5 : 1.0;
            val = fcq - 6.0 * w * (X * jx + Y * jy) * kk;
        } else {
            const double Mxx = cx ? PX[0] : PY[0];
            const double Myy = cy ? PY[2] : PX[2];
            const double Mxy = (cx && cy) ? PCxy : (cx ? PX[1] : PY[1]);
            const double eMe = X * X * Mxx + 2.0 * X * Y * Mxy + Y * Y * Myy;
            const double e2 = X * X + Y * Y;
            val = -fcq + 2.0 * w * (r0 + 0.5 * (9.0 * eMe - 3.0 * r0 * e2 - 3.0 * (Mxx + Myy) + 2.0 * r0));
        }
        fd[opp(q)] = val;
    }
}

// ---- step: interior nodes, y-marching ------------------------------------------------------
//
// Each wave owns the 64 columns [x0, x0 + 64), x0 = 64 s, of a strip and marches
// down a chunk of rows, so that every store covers whole cache lines (a partly
// written line costs a read-modify-write in HBM).  At iteration r it holds in
// registers the rows r..r+3 of u, r..r+2 of T, r-1..r+1 of sigma and r-1..r+1
// of the populations, and the loads of the rows D iterations ahead are in
// flight (D prefetch sets, so that no register holding a pending load is
// renamed; every iteration issues the same loads in the same order, so the
// waits stay counted; only the two rows that prime a chunk skip their stores).  x neighbours come from lane shifts, y
// neighbours from the rows held.
//
// What lanes 0 and 63 need from beyond the strip (u of x0-1 and x0+64, their
// T, and the pulled populations with their forcing) comes from a halo pass
// every HR rows: it gathers u on five columns per side, computes T on three,
// sigma and the six pull sources on the neighbour column, and leaves them in
// wave-private LDS (no barrier: only this wave reads them), where the lane
// shifts take them as the value shifted in at the edge.  The gathers of a
// halo pass are issued one block ahead.
//
// Waves whose rows and halo columns stay off the lattice edges (no clamping,
// wrapping or one-sided differences) run a copy of the loop without those
// selects.  Elsewhere, lanes beyond nx compute on clamped (or, periodic,
// wrapped) data and store into the row padding; the rows that prime a chunk
// store nothing.

template <typename T, typename TS, int HR>
struct Halo {  // rows k = 0..HR+5 of a block are rows r0 - 3 + k
    static constexpr int HK = HR + 6;
    double u[2][HK][5][2];  // [side][k][column c][comp]; side 0: x0-3+c, side 1: x0+62+c;
                            // iteration rel reads c = 2 of row r0 + rel + 2 (k = rel + 5)
    TS t[2][HK][3][4];      // T at c = 1, 2, 3
    TS s[2][HK][2];         // sigma at c = 2
    // what iteration rel of the block reads, side by side
    TS tn[2][HR][4];        // T at c = 2, row r0 + rel + 1
    T hn[2][HR][4];         // pull sources at c = 2: side 0 p = 1, 5, 8 from rows
                            // r0+rel, r0+rel-1, r0+rel+1; side 1 p = 3, 6, 7 likewise
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

template <bool B>
struct Flag {
    static constexpr bool value = B;
};

template <int PR, int HR>
using HaloOf = Halo<typename Store<PR>::T, typename Store<PR>::TS, HR>;

// One work item: rows [chk * chunk, chk * chunk + chunk) of the 64-column strip
// `strip` of the lattice a describes, by one wave (lane = its lane) with its
// LDS halo block hl.  PR: population storage; HR: rows per halo block; D: rows
// of loads in flight (prefetch sets).
template <int PR, int MAT, int HR, int D>
__device__ __forceinline__ void march_item(const StepArgs& a, HaloOf<PR, HR>& hl, int lane, int strip, int chk,
                                           int chunk) {
    using SF = Store<PR>;
    using T = typename SF::T;    // arithmetic type
    using TS = typename SF::TS;  // of the stresses and the source
    constexpr bool PK = SF::packed;
    // a row of one lane's populations as loaded: nine values, or five packed words
    using ST = typename SF::ST;
    using Raw = typename std::conditional<PK, uint32_t, ST>::type;
    constexpr int NRAW = PK ? 5 : 9;
    constexpr int HK = HR + 6;
    constexpr int L = (HR % D == 0) ? HR : (D % HR == 0 ? D : HR * D);  // iterations per loop trip
    // halo items per side: u of a whole block and of its new rows, T, sigma
    constexpr int NU = 5 * HK, NUN = 5 * HR, NT = 3 * (HK - 2), NS = HK - 4;
    static_assert(NU <= 64 && 2 * NT <= 64 && 2 * NS <= 64 && 6 * HR <= 64 && HR >= 1 && D >= 1,
                  "halo block too long for one wave");
    const Geometry g = a.g;
    const int x0 = strip * 64;
    const int vx = x0 + lane;  // this lane's column (< pitch)
    const int yc = chk * chunk, ye = min(yc + chunk, g.ny);
    const int ntrip = (ye - (yc - 2) + L - 1) / L;
    // rows and columns touched: rows yc-5 .. rmax, columns x0-3 .. x0+66
    const int rmax = yc + ntrip * L + 2 * HR + D + 4;
    const bool inner_y = g.py ? (yc - 5 >= 0 && rmax <= g.ny - 1) : (yc - 5 >= 1 && rmax <= g.ny - 2);
    const bool inner_x = g.px ? (x0 >= 3 && x0 + 66 <= g.nx - 1) : (x0 >= 4 && x0 + 66 <= g.nx - 2);

    // row records (u_at): u through one resource per buffer, its component rows
    // pbU bytes apart; the populations through a resource per lattice row, their
    // component rows pbF bytes apart (32-bit words: the 16-bit row at 4 pbF)
    const uint32_t pbU = (uint32_t)g.pitch * (uint32_t)sizeof(double);
    const uint32_t pbF = (uint32_t)g.pitch * (uint32_t)(PK ? 4 : sizeof(ST));
    const uint32_t recF = pop_row_bytes<PR>(g.pitch);
    const char* fs = reinterpret_cast<const char*>(a.fsrc);
    char* fd = reinterpret_cast<char*>(a.fdst);
    const uint32_t ubytes = (uint32_t)((size_t)g.plane * 2 * sizeof(double));
    const __amdgpu_buffer_rsrc_t rus = rsrc(a.usrc, ubytes), rud = rsrc(a.udst, ubytes);
    // Loads that no stored result needs go through empty ranges, so that they
    // return 0 and move no bytes while every loop trip issues the same loads:
    // the last trip's prefetch of populations beyond row ye and of u beyond row
    // ye + 2, and the halo gathers for the pass after the last block.  (8192^2
    // tension: FP32 +1.2 %, FP16 +0.7 %, FP64 -1 %, the compiler scheduling a
    // chunk's first loads differently; 1024^2 FP64, 4-row chunks, +18 %.)
    const __amdgpu_buffer_rsrc_t rnull = rsrc(a.usrc, 0u);
    // the record of lattice row y (wave-uniform) of a population buffer, or an
    // empty range (keep = false)
    auto frow = [&](const char* base, int y, bool keep) {
        return rsrc(base + (size_t)__builtin_amdgcn_readfirstlane(y) * recF, keep ? recF : 0u);
    };
    const T finv = T(a.k.finv), fscl = T(a.k.fscale);
    const double idx = a.k.inv_dx;
    const TS ic2 = TS(a.k.inv_c2), sbx = TS(a.k.sig_b[0]), sby = TS(a.k.sig_b[1]);
    const TS lam = TS(a.k.lam), mu = TS(a.k.mu);
    const double omd = a.k.omega;
    const CollideRates crk = collide_rates(omd, a.k.omega_p);
    const bool two_rates = a.k.omega_p != omd;

    auto run = [&](auto edge_flag, auto two_rates_flag) {
        constexpr bool EDGE = decltype(edge_flag)::value;
        constexpr bool TWO_RATES = decltype(two_rates_flag)::value;
        // row / column -> row / column to address: periodic wrap, else clamped
        auto rowp = [&](int r) -> int {
            if constexpr (EDGE) return g.py ? wrap(r, g.ny) : min(max(r, 0), g.ny - 1);
            else return r;
        };
        auto colp = [&](int c) -> int {
            if constexpr (EDGE) return g.px ? wrap(c, g.nx) : min(max(c, 0), g.nx - 1);
            else return c;
        };
        const int x = colp(vx);
        const bool xin = g.px || vx < g.nx;
        const bool atL = EDGE && xin && at_low(x, g.px), atR = EDGE && xin && at_high(x, g.nx, g.px);
        // one-sided differences at the lattice edges
        auto lo_row = [&](int r) { return EDGE && !g.py && r <= 0; };
        auto hi_row = [&](int r) { return EDGE && !g.py && r >= g.ny - 1; };

        auto load_u = [&](int r, double v[2]) {
            const uint32_t ob = (uint32_t)(rowp(r) * 2 * g.pitch + x) * (uint32_t)sizeof(double);
            const __amdgpu_buffer_rsrc_t ru = r <= ye + 2 ? rus : rnull;
            v[0] = bload(ru, ob, 0u, 0.0);
            v[1] = bload(ru, ob, pbU, 0.0);
        };
        // a row of populations as loaded (decoded only when consumed, so that the
        // loads stay in flight)
        auto load_f = [&](int r, Raw f[NRAW]) {
            const __amdgpu_buffer_rsrc_t rs = frow(fs, rowp(r), r <= ye);
            if constexpr (PK) {
#pragma unroll
                for (int w = 0; w < 4; w++)
                    f[w] = __builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)x * 4u, (uint32_t)w * pbF, 0);
                f[4] = __builtin_amdgcn_raw_buffer_load_b16(rs, (uint32_t)x * 2u, 4u * pbF, 0);
            } else {
                const uint32_t ob = (uint32_t)x * (uint32_t)sizeof(ST);
#pragma unroll
                for (int q = 0; q < 9; q++) f[q] = bload(rs, ob, (uint32_t)q * pbF, ST(0));
            }
        };
        auto decode = [&](const Raw f[NRAW], T F[9]) {
            if constexpr (PK) {
#pragma unroll
                for (int w = 0; w < 4; w++) {
                    F[2 * w] = SF::dec(f[w]) * finv;
                    F[2 * w + 1] = SF::dec(f[w] >> 16) * finv;
                }
                F[8] = SF::dec(f[4]) * finv;
            } else {
#pragma unroll
                for (int q = 0; q < 9; q++) F[q] = T(f[q]);
            }
        };
        // the new state of this lane's node (column vx) of row r (wave-uniform)
        auto store_node = [&](int r, double ux, double uy, const T fn[9]) {
            const uint32_t ou = (uint32_t)(r * 2 * g.pitch + vx) * (uint32_t)sizeof(double);
            bstore_nt(rud, ou, 0u, ux);
            bstore_nt(rud, ou, pbU, uy);
            const __amdgpu_buffer_rsrc_t rd = frow(fd, r, true);
            if constexpr (PK) {
#pragma unroll
                for (int w = 0; w < 4; w++)
                    __builtin_amdgcn_raw_buffer_store_b32(
                        SF::enc(fn[2 * w] * fscl) | (SF::enc(fn[2 * w + 1] * fscl) << 16), rd, (uint32_t)vx * 4u,
                        (uint32_t)w * pbF, kCpolNT);
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)SF::enc(fn[8] * fscl), rd, (uint32_t)vx * 2u,
                                                      4u * pbF, kCpolNT);
            } else {
                const uint32_t of = (uint32_t)vx * (uint32_t)sizeof(ST);
#pragma unroll
                for (int q = 0; q < 9; q++) bstore_nt(rd, of, (uint32_t)q * pbF, ST(fn[q]));
            }
        };

        // T = P(H) + Pi(H) at row r of this lane; ul / ur: u of the columns left of
        // lane 0 and right of lane 63
        auto stress = [&](int r, const double um[2], const double u0[2], const double up[2], auto* t,
                          const double ul[2], const double ur[2]) {
            using TT = typename std::remove_pointer<decltype(t)>::type;  // TS, or double at walls
            double lx = from_prev(u0[0], ul[0]), rx = from_next(u0[0], ur[0]);
            double ly = from_prev(u0[1], ul[1]), ry = from_next(u0[1], ur[1]);
            double fx = 0.5 * idx, fy = 0.5 * idx;
            double cx = um[0], dx = up[0], cy = um[1], dy = up[1];
            if constexpr (EDGE) {
                lx = atL ? u0[0] : lx;
                ly = atL ? u0[1] : ly;
                rx = atR ? u0[0] : rx;
                ry = atR ? u0[1] : ry;
                fx = (atL || atR) ? idx : fx;
                const bool lo = lo_row(r), hi = hi_row(r);
                cx = lo ? u0[0] : cx;
                cy = lo ? u0[1] : cy;
                dx = hi ? u0[0] : dx;
                dy = hi ? u0[1] : dy;
                fy = (lo || hi) ? idx : fy;
            }
            excess_stress<TT, MAT>(TT((rx - lx) * fx), TT((dx - cx) * fy), TT((ry - ly) * fx),
                                   TT((dy - cy) * fy), TT(a.k.lam), TT(a.k.mu), t);
        };
        // sigma = dt S / c at row r of this lane; tl / tr: T of the columns left of
        // lane 0 and right of lane 63
        auto sigma = [&](int r, const auto* tm, const auto* t0, const auto* tp, TS sg[2], const TS tl[4],
                         const TS tr[4]) {
            using TT = typename std::remove_cv<typename std::remove_pointer<decltype(t0)>::type>::type;
            TT lxx = from_prev(t0[0], TT(tl[0])), rxx = from_next(t0[0], TT(tr[0]));
            TT lyx = from_prev(t0[2], TT(tl[2])), ryx = from_next(t0[2], TT(tr[2]));
            TT fx = TT(0.5), fy = TT(0.5);
            TT cxy = tm[1], dxy = tp[1], cyy = tm[3], dyy = tp[3];
            if constexpr (EDGE) {
                lxx = atL ? t0[0] : lxx;
                lyx = atL ? t0[2] : lyx;
                rxx = atR ? t0[0] : rxx;
                ryx = atR ? t0[2] : ryx;
                fx = (atL || atR) ? TT(1) : fx;
                const bool lo = lo_row(r), hi = hi_row(r);
                cxy = lo ? t0[1] : cxy;
                cyy = lo ? t0[3] : cyy;
                dxy = hi ? t0[1] : dxy;
                dyy = hi ? t0[3] : dyy;
                fy = (lo || hi) ? TT(1) : fy;
            }
            sg[0] = TS(TT(ic2) * ((rxx - lxx) * fx + (dxy - cxy) * fy) + TT(sbx));
            sg[1] = TS(TT(ic2) * ((ryx - lyx) * fx + (dyy - cyy) * fy) + TT(sby));
        };

        // ---- halo: gathers (issued one block ahead) and the pass that fills the LDS
        //
        // A block's rows k = 0..5 are rows HR..HR+5 of the block before, so after the
        // first block of a chunk only the HR new rows of u are gathered and the rest
        // is moved within the LDS.  Each pulled population is gathered on the HR rows
        // whose pulls use it (pull i of row rel comes from row rel + hrow(i)).
        double gu[2][2];  // u gathered for the next halo pass: [side][comp]
        Raw gf;           // population gathered for it (raw; packed: the word holding it)
        // lane j < 6 HR: the halo population of side j / (3 HR), pull (j / HR) % 3, row j % HR
        auto hrow = [](int pi) { return pi == 0 ? 3 : (pi == 1 ? 2 : 4); };  // its block row k - rel
        // where this lane's halo population sits in a packed word: the high half?
        // (population 8: the parity of its column, as every row of a record starts
        // at an even 16-bit unit)
        const bool ghigh = [&] {
            const int j = min(lane, 6 * HR - 1);
            const int sd = j / (3 * HR);
            const int p = halo_pop(sd, (j % (3 * HR)) / HR);
            const int hx = colp(sd == 0 ? x0 - 1 : x0 + 64);
            return p == 8 ? (hx & 1) != 0 : (p & 1) != 0;
        }();
        // u: all rows of the block (full, the first block of a chunk) or its new ones
        // used = false: a gather no halo pass consumes (u from the empty range,
        // the population from the buffer's first word)
        auto gather = [&](int r0, bool full, bool used) {
            const int i = min(lane, (full ? NU : NUN) - 1);
            const int c = i % 5, k = (full ? 0 : 6) + i / 5;
            const int rr = rowp(r0 - 3 + k);
            const __amdgpu_buffer_rsrc_t rg = used ? rus : rnull;
#pragma unroll
            for (int sd = 0; sd < 2; sd++) {
                const int hx = colp(sd == 0 ? x0 - 3 + c : x0 + 62 + c);
                const uint32_t ob = (uint32_t)(rr * 2 * g.pitch + hx) * (uint32_t)sizeof(double);
                gu[sd][0] = bload(rg, ob, 0u, 0.0);
                gu[sd][1] = bload(rg, ob, pbU, 0.0);
            }
            const int j = min(lane, 6 * HR - 1);
            const int sd = j / (3 * HR), pi = (j % (3 * HR)) / HR, k2 = j % HR + hrow(pi);
            const int hx = colp(sd == 0 ? x0 - 1 : x0 + 64);
            const int p = halo_pop(sd, pi);
            const size_t gy = (size_t)rowp(r0 - 3 + k2);
            if constexpr (PK) {
                // population 8 from the 32-bit word of its 16-bit row that holds it
                const uint32_t* w = reinterpret_cast<const uint32_t*>(fs);
                const size_t row = gy * 9 * (size_t)g.pitch;  // the record's first 16-bit unit
                const size_t wi = p == 8 ? (row + 8 * (size_t)g.pitch + hx) >> 1 : row / 2 + (size_t)(p >> 1) * g.pitch + hx;
                gf = w[used ? wi : 0];
            } else {
                const size_t ei = (gy * 9 + p) * g.pitch + hx;
                gf = reinterpret_cast<const ST*>(fs)[used ? ei : 0];
            }
        };
        auto halo = [&](int r0, bool full) {
            wave_lds_sync();  // the last block's reads come first
            if (full) {
                if (lane < NU) {
                    const int c = lane % 5, k = lane / 5;
#pragma unroll
                    for (int sd = 0; sd < 2; sd++) {
                        hl.u[sd][k][c][0] = gu[sd][0];
                        hl.u[sd][k][c][1] = gu[sd][1];
                    }
                }
            } else {
                // rows HR..HR+5 of the last block become rows 0..5 (every lane reads
                // before any lane writes: one LDS read, then the writes, in order)
                double mv[2][2];
                const int c = lane % 5, k = lane / 5;
                if (lane < 30) {
#pragma unroll
                    for (int sd = 0; sd < 2; sd++) {
                        mv[sd][0] = hl.u[sd][k + HR][c][0];
                        mv[sd][1] = hl.u[sd][k + HR][c][1];
                    }
                }
                wave_lds_sync();
                if (lane < 30) {
#pragma unroll
                    for (int sd = 0; sd < 2; sd++) {
                        hl.u[sd][k][c][0] = mv[sd][0];
                        hl.u[sd][k][c][1] = mv[sd][1];
                    }
                }
                if (lane < NUN) {
#pragma unroll
                    for (int sd = 0; sd < 2; sd++) {
                        hl.u[sd][6 + k][c][0] = gu[sd][0];
                        hl.u[sd][6 + k][c][1] = gu[sd][1];
                    }
                }
            }
            wave_lds_sync();
            if (lane < 2 * NT) {  // T at c = 1, 2, 3 and k = 1..HK-2, both sides
                const int sd = lane / NT, jj = lane % NT, c = 1 + jj % 3, k = 1 + jj / 3;
                const int X = colp(sd == 0 ? x0 - 3 + c : x0 + 62 + c);
                const int r = r0 - 3 + k;
                const double u0x = hl.u[sd][k][c][0], u0y = hl.u[sd][k][c][1];
                const bool aL = EDGE && !g.px && X == 0, aR = EDGE && !g.px && X == g.nx - 1;
                const double ax = aL ? u0x : hl.u[sd][k][c - 1][0], bx = aR ? u0x : hl.u[sd][k][c + 1][0];
                const double ay = aL ? u0y : hl.u[sd][k][c - 1][1], by = aR ? u0y : hl.u[sd][k][c + 1][1];
                const double fx = (aL || aR) ? idx : 0.5 * idx;
                const bool lo = lo_row(r), hi = hi_row(r);
                const double cx = lo ? u0x : hl.u[sd][k - 1][c][0], dx = hi ? u0x : hl.u[sd][k + 1][c][0];
                const double cy = lo ? u0y : hl.u[sd][k - 1][c][1], dy = hi ? u0y : hl.u[sd][k + 1][c][1];
                const double fy = (lo || hi) ? idx : 0.5 * idx;
                TS t[4];
                excess_stress<TS, MAT>(TS((bx - ax) * fx), TS((dx - cx) * fy), TS((by - ay) * fx),
                                       TS((dy - cy) * fy), lam, mu, t);
#pragma unroll
                for (int q = 0; q < 4; q++) hl.t[sd][k][c - 1][q] = t[q];
                // T at c = 2 for the iteration that needs it: row r0 + rel + 1, k = rel + 4
                if (c == 2 && k >= 4 && k < 4 + HR) {
#pragma unroll
                    for (int q = 0; q < 4; q++) hl.tn[sd][k - 4][q] = t[q];
                }
            }
            wave_lds_sync();
            if (lane < 2 * NS) {  // sigma at c = 2 and k = 2..HK-3
                const int sd = lane / NS, k = 2 + lane % NS;
                const int X = colp(sd == 0 ? x0 - 1 : x0 + 64);
                const int r = r0 - 3 + k;
                const bool aL = EDGE && !g.px && X == 0, aR = EDGE && !g.px && X == g.nx - 1;
                const TS t0xx = hl.t[sd][k][1][0], t0yx = hl.t[sd][k][1][2];
                const TS axx = aL ? t0xx : hl.t[sd][k][0][0], bxx = aR ? t0xx : hl.t[sd][k][2][0];
                const TS ayx = aL ? t0yx : hl.t[sd][k][0][2], byx = aR ? t0yx : hl.t[sd][k][2][2];
                const TS fx = (aL || aR) ? TS(1) : TS(0.5);
                const bool lo = lo_row(r), hi = hi_row(r);
                const TS cxy = lo ? hl.t[sd][k][1][1] : hl.t[sd][k - 1][1][1];
                const TS dxy = hi ? hl.t[sd][k][1][1] : hl.t[sd][k + 1][1][1];
                const TS cyy = lo ? hl.t[sd][k][1][3] : hl.t[sd][k - 1][1][3];
                const TS dyy = hi ? hl.t[sd][k][1][3] : hl.t[sd][k + 1][1][3];
                const TS fy = (lo || hi) ? TS(1) : TS(0.5);
                hl.s[sd][k][0] = ic2 * ((bxx - axx) * fx + (dxy - cxy) * fy) + sbx;
                hl.s[sd][k][1] = ic2 * ((byx - ayx) * fx + (dyy - cyy) * fy) + sby;
            }
            wave_lds_sync();
            if (lane < 6 * HR) {  // pull sources: the population plus dt psi at the source
                const int sd = lane / (3 * HR), pi = (lane % (3 * HR)) / HR, rel = lane % HR, k = rel + hrow(pi);
                const int p = halo_pop(sd, pi);
                T fp;
                if constexpr (PK) fp = SF::dec(ghigh ? (gf >> 16) : gf) * finv;
                else fp = T(gf);
                const T hv = fp + T(3) * wq<T>(p) * T(TS(ex(p)) * hl.s[sd][k][0] + TS(ey(p)) * hl.s[sd][k][1]);
                // the iteration pulling it: p = 1, 3 from its own row (k = rel + 3),
                // p = 5, 6 from the row before (k = rel + 2), p = 7, 8 from the row after
                hl.hn[sd][rel][pi] = hv;
            }
            wave_lds_sync();
        };

        // ---- the row pipeline
        double U0[2], U1[2], U2[2], tmp[2];
        TS T0[4], T1[4];
        TS Gm[2] = {TS(0), TS(0)}, G0[2] = {TS(0), TS(0)};
        T Fm[9], F0[9];
        // rows of loads in flight: the FP64 edge path keeps one, which leaves the
        // registers its wall rules need (its waves are a few percent of the grid)
        constexpr int DD = (EDGE && sizeof(T) == 8) ? 1 : D;
        static_assert(L % DD == 0, "prefetch sets must divide the loop trip");
        double UP[DD][2];
        Raw FP[DD][NRAW];

        // iteration r, the block's relative row rel (0..HR-1)
        auto iteration = [&](int r, int rel, double Us[2], Raw Fs[NRAW]) {
            double U3[2] = {Us[0], Us[1]};
            T F1[9];
            decode(Fs, F1);
            load_u(r + 3 + DD, Us);
            load_f(r + 1 + DD, Fs);
            const double ul[2] = {hl.u[0][rel + 5][2][0], hl.u[0][rel + 5][2][1]};
            const double ur[2] = {hl.u[1][rel + 5][2][0], hl.u[1][rel + 5][2][1]};
            TS T2[4], G1[2];
            stress(r + 2, U1, U2, U3, T2, ul, ur);
            TS tl[4], tr[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                tl[q] = hl.tn[0][rel][q];
                tr[q] = hl.tn[1][rel][q];
            }
            sigma(r + 1, T0, T1, T2, G1, tl, tr);

            T h[9];
            h[0] = F0[0];
            h[1] = F0[1] + T(3) * wq<T>(1) * T(G0[0]);
            h[3] = F0[3] - T(3) * wq<T>(3) * T(G0[0]);
            h[2] = Fm[2] + T(3) * wq<T>(2) * T(Gm[1]);
            h[5] = Fm[5] + T(3) * wq<T>(5) * T(Gm[0] + Gm[1]);
            h[6] = Fm[6] + T(3) * wq<T>(6) * T(Gm[1] - Gm[0]);
            h[4] = F1[4] - T(3) * wq<T>(4) * T(G1[1]);
            h[7] = F1[7] - T(3) * wq<T>(7) * T(G1[0] + G1[1]);
            h[8] = F1[8] + T(3) * wq<T>(8) * T(G1[0] - G1[1]);
            T hL[4], hR[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                hL[q] = hl.hn[0][rel][q];
                hR[q] = hl.hn[1][rel][q];
            }
            T f[9];
            f[0] = h[0];
            f[2] = h[2];
            f[4] = h[4];
            f[1] = from_prev(h[1], hL[0]);
            f[5] = from_prev(h[5], hL[1]);
            f[8] = from_prev(h[8], hL[2]);
            f[3] = from_next(h[3], hR[0]);
            f[6] = from_next(h[6], hR[1]);
            f[7] = from_next(h[7], hR[2]);
            // Moments, equilibrium and relaxation in FP64 in every mode: the D2Q9
            // weights are not exact in FP32 (3 (2 w1 + 4 w5) rounds to 1 + 7.5e-9),
            // so an FP32 equilibrium scales j and Pi by about 1 + omega 7.5e-9 in
            // every collision, a bias that compounds over the steps.
            double fd[9], fnd[9];
#pragma unroll
            for (int q = 0; q < 9; q++) fd[q] = (double)f[q];
            const NodeMoments mo = collide_node<TWO_RATES>(fd, crk, fnd);
            const double m1x = mo.m1x, m1y = mo.m1y;
            // first moment of the node's own populations before streaming (j_n)
            const double g57 = (double)F0[5] - (double)F0[7], g86 = (double)F0[8] - (double)F0[6];
            const double o1x = ((double)F0[1] - (double)F0[3]) + (g57 + g86);
            const double o1y = ((double)F0[2] - (double)F0[4]) + (g57 - g86);
            T fn[9];
#pragma unroll
            for (int q = 0; q < 9; q++) fn[q] = T(fnd[q]);
            // the two rows that prime the chunk store nothing, and nor do the
            // rows and lanes on non-periodic sides: the wall blocks of the same
            // launch write those nodes (rows wave-uniform; lanes only in the
            // edge copy of the loop)
            if (r >= yc && r < ye && !lo_row(r) && !hi_row(r) && !atL && !atR)
                store_node(r, U0[0] + a.k.ucoef * (m1x + o1x + (double)G0[0]),
                           U0[1] + a.k.ucoef * (m1y + o1y + (double)G0[1]), fn);

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
        // rows, the prefetch sets and the gathers of the next block, in the order
        // the loop repeats
        int r0 = yc - 2;
        gather(r0, true, true);
        halo(r0, true);
        load_u(yc - 3, tmp);
        load_u(yc - 2, U0);
        load_u(yc - 1, U1);
        load_u(yc, U2);
#pragma unroll
        for (int i = 0; i < DD; i++) {
            load_u(yc + 1 + i, UP[i]);
            load_f(yc - 1 + i, FP[i]);
        }
        gather(r0 + HR, false, true);
        {
            // T of the rows yc-2 (k = 3) and yc-1 (k = 4) of the first block
            const double l3[2] = {hl.u[0][3][2][0], hl.u[0][3][2][1]}, r3[2] = {hl.u[1][3][2][0], hl.u[1][3][2][1]};
            const double l4[2] = {hl.u[0][4][2][0], hl.u[0][4][2][1]}, r4[2] = {hl.u[1][4][2][0], hl.u[1][4][2][1]};
            stress(yc - 2, tmp, U0, U1, T0, l3, r3);
            stress(yc - 1, U0, U1, U2, T1, l4, r4);
        }

#pragma unroll
        for (int q = 0; q < 9; q++) { Fm[q] = T(0); F0[q] = T(0); }

        // the loop's halo passes: pass h prepares block h + 1, the gather issued
        // with it feeds pass h + 1
        constexpr int HPT = L / HR;
        const int nhalo = ntrip * HPT;
        for (int b = 0; b < ntrip; b++) {
#pragma unroll
            for (int j = 0; j < L; j++) {
                iteration(r0 + j % HR, j % HR, UP[j % DD], FP[j % DD]);
                if (j % HR == HR - 1) {
                    r0 += HR;
                    halo(r0, false);
                    gather(r0 + HR, false, b * HPT + j / HR + 2 < nhalo);
                }
            }
        }
    };
    // copies of the loop: edge or interior, BGK or two relaxation times
    if (inner_x && inner_y) {
        if (two_rates) run(Flag<false>{}, Flag<true>{});
        else run(Flag<false>{}, Flag<false>{});
    } else {
        if (two_rates) run(Flag<true>{}, Flag<true>{});
        else run(Flag<true>{}, Flag<false>{});
    }
}

// ---- per-node helpers for init, read-out, diagnostics and the multi-pass step (FP64) -------

__device__ __forceinline__ double ld_u(const InitLike& a, int c, int gx, int gy) {
    return a.u[u_at(a.g, c, gy, gx)];
}

// Difference of a field along one axis at index m (0..n-1) of that axis, times
// h (the spacing): central (v+ - v-) / 2 inside and across a periodic wrap;
// at the outermost nodes of a non-periodic axis one-sided with the inward
// neighbours, first order s (v1 - v0) or second order s (-3 v0 + 4 v1 - v2) / 2,
// s = +1 at the low end, -1 at the high end (Sect. 3.2).  get(k) reads the
// field at axis index k.
template <typename Get>
__device__ __forceinline__ double axis_diff(Get get, int m, int n, int per, int bo) {
    if (per) return 0.5 * (get(wrap1(m + 1, n)) - get(wrap1(m - 1, n)));
    if (m == 0 || m == n - 1) {
        const int s = m == 0 ? 1 : -1;
        if (bo == 2) return s * (-3.0 * get(m) + 4.0 * get(m + s) - get(m + 2 * s)) * 0.5;
        return s * (get(m + s) - get(m));
    }
    return 0.5 * (get(m + 1) - get(m - 1));
}

// H = grad u at a node, (xx, xy, yx, yy)
__device__ void node_H(const InitLike& a, int gx, int gy, double H[4]) {
    const Geometry& g = a.g;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        H[2 * c] = axis_diff([&](int k) { return ld_u(a, c, k, gy); }, gx, g.nx, g.px, a.bo) * a.inv_dx;
        H[2 * c + 1] = axis_diff([&](int k) { return ld_u(a, c, gx, k); }, gy, g.ny, g.py, a.bo) * a.inv_dx;
    }
}

template <int MAT>
__device__ void node_T(const InitLike& a, int gx, int gy, double t[4]) {
    double H[4];
    node_H(a, gx, gy, H);
    excess_stress<double, MAT>(H[0], H[1], H[2], H[3], a.lam, a.mu, t);
}

// sigma = dt S / c at a node, from T at the nodes a get(x, y, t) supplies
template <typename GetT>
__device__ void sigma_from(const InitLike& a, int gx, int gy, GetT getT, double s[2]) {
    const Geometry& g = a.g;
    double d[2][2];  // d[row a][axis b] = dT_ab along b (times dX)
#pragma unroll
    for (int r = 0; r < 2; r++) {
        d[r][0] = axis_diff([&](int k) { double t[4]; getT(k, gy, t); return t[2 * r]; }, gx, g.nx, g.px, a.bo);
        d[r][1] = axis_diff([&](int k) { double t[4]; getT(gx, k, t); return t[2 * r + 1]; }, gy, g.ny, g.py, a.bo);
    }
    s[0] = a.inv_c2 * (d[0][0] + d[0][1]) + a.sig_b[0];
    s[1] = a.inv_c2 * (d[1][0] + d[1][1]) + a.sig_b[1];
}

template <int MAT>
__device__ void node_sigma(const InitLike& a, int gx, int gy, double s[2]) {
    sigma_from(a, gx, gy, [&](int x, int y, double t[4]) { node_T<MAT>(a, x, y, t); }, s);
}

// ---- init ------------------------------------------------------------------------------

// fc'_0 = f_eq(r0 = -rho0 tr H(u0), j0, Pi(H(u0))): an equilibrium is unchanged by
// the collision without forcing.
template <int PR>
__global__ __launch_bounds__(256) void init_kernel(InitArgs a) {
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (gx >= a.b.g.nx || gy >= a.b.g.ny) return;
    double H[4];
    node_H(a.b, gx, gy, H);
    const double tr = H[0] + H[3];
    const double r0 = -a.rho0 * tr;
    const double ic2 = a.b.inv_c2;
    const double m2xx = -a.b.mu * (H[0] + H[0] + tr) * ic2;
    const double m2xy = -a.b.mu * (H[1] + H[2]) * ic2;
    const double m2yy = -a.b.mu * (H[3] + H[3] + tr) * ic2;
    const double m1x = a.j0[u_at(a.b.g, 0, gy, gx)] * a.inv_c, m1y = a.j0[u_at(a.b.g, 1, gy, gx)] * a.inv_c;
    double v[9];
#pragma unroll
    for (int q = 0; q < 9; q++) v[q] = feq_q<double>(q, r0, m1x, m1y, m2xx, m2xy, m2yy);
    pop_put_all<PR>(a.f, a.b.g, gy, gx, v, a.fscale);
}

// ---- read-out -----------------------------------------------------------------------------

// sigma of the collision at t_n: held (the printed order's level n - 1) or from u_n
template <int MAT>
__device__ __forceinline__ void collision_sigma(const ReadArgs& a, int gx, int gy, double s[2]) {
    if (a.sig) {
        const size_t o = (size_t)gy * a.b.g.pitch + gx;
        s[0] = a.sig[o];
        s[1] = a.sig[(size_t)a.b.g.plane + o];
    } else {
        node_sigma<MAT>(a.b, gx, gy, s);
    }
}

template <int PR, int MAT>
__global__ __launch_bounds__(256) void read_kernel(ReadArgs a) {
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    const Geometry& g = a.b.g;
    if (gx >= g.nx || gy >= g.ny) return;
    const size_t oc = (size_t)gy * g.nx + gx, pc = (size_t)g.nx * g.ny;  // compact output
    double* d = a.dst;
    // component c of the field goes to plane c - c0 when c0 <= c < c1
    auto put = [&](int c, double v) {
        if (c >= a.c0 && c < a.c1) d[(size_t)(c - a.c0) * pc + oc] = v;
    };
    switch (a.field) {
    case 0:  // U
        put(0, a.b.u[u_at(g, 0, gy, gx)]);
        put(1, a.b.u[u_at(g, 1, gy, gx)]);
        break;
    case 1: {  // J = c (M1' + sigma / 2)
        double s[2], mx = 0, my = 0;
        collision_sigma<MAT>(a, gx, gy, s);
        for (int q = 0; q < 9; q++) {
            const double v = pop_get<PR>(a.f, g, gy, gx, q, a.finv);
            mx += ex(q) * v;
            my += ey(q) * v;
        }
        put(0, a.c * (mx + 0.5 * s[0]));
        put(1, a.c * (my + 0.5 * s[1]));
        break;
    }
    case 2:  // R
    case 3: {  // PI = c^2 M2'
        double r = 0, pxx = 0, pxy = 0, pyy = 0;
        for (int q = 0; q < 9; q++) {
            const double v = pop_get<PR>(a.f, g, gy, gx, q, a.finv);
            r += v;
            pxx += ex(q) * ex(q) * v;
            pxy += ex(q) * ey(q) * v;
            pyy += ey(q) * ey(q) * v;
        }
        if (a.field == 2) {
            put(0, r);
        } else {
            const double c2 = a.c * a.c;
            put(0, c2 * pxx);
            put(1, c2 * pxy);
            put(2, c2 * pyy);
        }
        break;
    }
    case 4:  // H
    case 5: {  // P
        double H[4], P[4];
        node_H(a.b, gx, gy, H);
        if (a.field == 5) first_pk<double, MAT>(H[0], H[1], H[2], H[3], a.b.lam, a.b.mu, P);
        for (int c = 0; c < 4; c++) put(c, a.field == 4 ? H[c] : P[c]);
        break;
    }
    case 6: {  // S (from u_n)
        double s[2];
        node_sigma<MAT>(a.b, gx, gy, s);
        put(0, s[0] * a.s_from_sig);
        put(1, s[1] * a.s_from_sig);
        break;
    }
    default: break;
    }
}

// ---- diagnostics: fixed-order reductions (wavefront lane shifts, then blocks) ----------------------

// sum or max of v over the 64 lanes of this wave, in a fixed order (butterfly
// through lane shuffles); every lane receives the result
__device__ __forceinline__ double wave_reduce(double v, bool take_max) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = take_max ? fmax(v, o) : v + o;
    }
    return v;
}

// the diagnostics of one node: momentum x, y, kinetic energy, |u|^2, non-finite
template <int PR, int MAT>
__device__ __forceinline__ void diag_node(const ReadArgs& a, int gx, int gy, double v[5]) {
    const Geometry& g = a.b.g;
    double mx = 0, my = 0, s[2];
    for (int q = 0; q < 9; q++) {
        const double w = pop_get<PR>(a.f, g, gy, gx, q, a.finv);
        mx += ex(q) * w;
        my += ey(q) * w;
    }
    collision_sigma<MAT>(a, gx, gy, s);
    const double jx = a.c * (mx + 0.5 * s[0]), jy = a.c * (my + 0.5 * s[1]);
    const double ux = a.b.u[u_at(g, 0, gy, gx)], uy = a.b.u[u_at(g, 1, gy, gx)];
    v[0] = a.c * mx;
    v[1] = a.c * my;
    v[2] = (jx * jx + jy * jy) / (2.0 * a.b.rho0);
    v[3] = ux * ux + uy * uy;
    v[4] = (isfinite(jx) && isfinite(jy) && isfinite(ux) && isfinite(uy)) ? 0.0 : 1.0;
    if (v[4] != 0.0) v[3] = 0.0;
}

// Tiles of 64 x 4 nodes; block b takes the tiles b, b + grid, ... (one tile per
// block when the grid has one block per tile), and writes its partial sums
// (maxima for |u|^2 and the flag) to partial[8 b ..]: a fixed order, so the
// result is deterministic for a given grid.
template <int PR, int MAT>
__global__ __launch_bounds__(256) void diag_kernel(ReadArgs a) {
    const Geometry& g = a.b.g;
    const int nbx = (g.nx + 63) / 64, ntiles = nbx * ((g.ny + 3) / 4);
    double v[5] = {0, 0, 0, 0, 0};  // momentum x, y, ekin, max |u|^2, non-finite
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int bx = tile % nbx, by = tile / nbx;
        const int gx = bx * 64 + (threadIdx.x & 63), gy = by * 4 + (threadIdx.x >> 6);
        if (gx < g.nx && gy < g.ny) {
            double w[5];
            diag_node<PR, MAT>(a, gx, gy, w);
            v[0] += w[0];
            v[1] += w[1];
            v[2] += w[2];
            v[3] = fmax(v[3], w[3]);
            v[4] = fmax(v[4], w[4]);
        }
    }
    // each wave reduces its 64 lanes with lane shifts, then the block's four
    // wave results are added in wave order
    __shared__ double red[4][5];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 5; c++) {
        const double r = wave_reduce(v[c], c >= 3);
        if (lane == c) red[wv][c] = r;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int c = threadIdx.x;
        double r = red[0][c];
        for (int w = 1; w < 4; w++) r = (c >= 3) ? fmax(r, red[w][c]) : r + red[w][c];
        a.partial[(size_t)blockIdx.x * 8 + c] = r;
    }
}

// the block partials into out[0..4]; with watch set, lane 0 also records step in
// watch[0] when the totals are not finite and watch[0] is still -1 (a vector
// store from one lane)
__global__ __launch_bounds__(256) void diag_reduce_kernel(const double* partial, int nblk, double* out,
                                                          int64_t* watch, int64_t step) {
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256)
        for (int c = 0; c < 5; c++) {
            const double x = partial[(size_t)b * 8 + c];
            v[c] = (c == 3 || c == 4) ? fmax(v[c], x) : v[c] + x;
        }
    __shared__ double red[4][5];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 5; c++) {
        const double r = wave_reduce(v[c], c >= 3);
        if (lane == c) red[wv][c] = r;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int c = threadIdx.x;
        double r = red[0][c];
        for (int w = 1; w < 4; w++) r = (c >= 3) ? fmax(r, red[w][c]) : r + red[w][c];
        out[c] = r;
        if (watch && c == 4 && r != 0.0 && watch[0] < 0) watch[0] = step;
    }
}

// ---- the multi-pass step: second-order boundary differences, the printed time order -------
//
// Three launches per step, per node and in FP64 whatever the storage:
//   1. stress pass: T_n = P(H) + Pi(H) from u_n (boundary differences of order bo)
//   2. source pass: sigma_n = dt S_n / c from T_n (same differences)
//   3. step: pull f(t_{n+1})_q = fc'_q(X - e_q) + dt psi_q(sigma_c(X - e_q)), the
//      wall rules with the stresses Tw, u_{n+1} = u_n + dt/(2 rho0)(j_{n+1} + j_n)
//      with j_n = c (M1(fc'_n) + sigma_c / 2) and j_{n+1} = c (M1(f) + sigma_n / 2),
//      and the collision to fc'_{n+1}.
// At the current level (Sect. 3.1) sigma_c = sigma_n and Tw = T_n; in the order
// printed in Algorithm 1 they are the held sigma_{n-1} and T_{n-1}.

template <int MAT>
__global__ __launch_bounds__(256) void stress_pass_kernel(InitLike b, double* T) {
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (gx >= b.g.nx || gy >= b.g.ny) return;
    const size_t plane = (size_t)b.g.plane, o = (size_t)gy * b.g.pitch + gx;
    double t[4];
    node_T<MAT>(b, gx, gy, t);
#pragma unroll
    for (int c = 0; c < 4; c++) T[(size_t)c * plane + o] = t[c];
}

__global__ __launch_bounds__(256) void source_pass_kernel(InitLike b, const double* __restrict__ T,
                                                          double* __restrict__ sig) {
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (gx >= b.g.nx || gy >= b.g.ny) return;
    const size_t plane = (size_t)b.g.plane, o = (size_t)gy * b.g.pitch + gx;
    double s[2];
    sigma_from(b, gx, gy,
               [&](int x, int y, double t[4]) {
                   const size_t oo = (size_t)y * b.g.pitch + x;
#pragma unroll
                   for (int c = 0; c < 4; c++) t[c] = T[(size_t)c * plane + oo];
               },
               s);
    sig[o] = s[0];
    sig[plane + o] = s[1];
}

// The displacement and constants of a step, for the per-node helpers.
__device__ __forceinline__ InitLike init_like(const StepArgs& a, int bo) {
    InitLike b;
    b.u = a.usrc;
    b.g = a.g;
    b.inv_dx = a.k.inv_dx;
    b.inv_c2 = a.k.inv_c2;
    b.sig_b[0] = a.k.sig_b[0];
    b.sig_b[1] = a.k.sig_b[1];
    b.lam = a.k.lam;
    b.mu = a.k.mu;
    b.rho0 = a.k.rho0;
    b.bo = bo;
    return b;
}

// The whole update of one node in FP64, walls included: pull
// f(t_{n+1})_q = fc'_q(X - e_q) + dt psi_q(sigma_c(X - e_q)), the wall rules
// (apply_walls) with the stresses Tw, u_{n+1} = u_n + dt/(2 rho0)(j_{n+1} + j_n)
// with j_n = c (M1(fc'_n) + sigma_c / 2) and j_{n+1} = c (M1(f) + sigma_n / 2),
// and the collision to fc'_{n+1}.  sig_c(x, y, s): sigma of the collision at
// t_n at a node; sig_n(s): sigma_n at this node; Tw(x, y, t): the stresses the
// walls use.
template <int PR, bool TWO_RATES, typename SigC, typename SigN, typename TW>
__device__ __forceinline__ void node_update(const StepArgs& a, int gx, int gy, SigC sig_c, SigN sig_n, TW Tw) {
    const Geometry& g = a.g;
    const double finv = a.k.finv;
    double fo[9], f[9];
#pragma unroll
    for (int q = 0; q < 9; q++) fo[q] = pop_get<PR>(a.fsrc, g, gy, gx, q, finv);
    // pulls with the forcing of the collision at the source node
#pragma unroll
    for (int q = 0; q < 9; q++) {
        int sx = gx - ex(q), sy = gy - ey(q);
        if (g.px) sx = wrap1(sx, g.nx);
        if (g.py) sy = wrap1(sy, g.ny);
        f[q] = 0.0;  // links from beyond a wall: the wall rules below
        if (sx < 0 || sx >= g.nx || sy < 0 || sy >= g.ny) continue;
        double sg[2];
        sig_c(sx, sy, sg);
        f[q] = pop_get<PR>(a.fsrc, g, sy, sx, q, finv) +
               3.0 * wq<double>(q) * (ex(q) * sg[0] + ey(q) * sg[1]);
    }
    const bool atL = !g.px && gx == 0, atR = !g.px && gx == g.nx - 1;
    const bool wyB = !g.py && gy == 0, wyT = !g.py && gy == g.ny - 1;
    double sc[2];
    sig_c(gx, gy, sc);
    if (atL || atR || wyB || wyT) {
        double td[4], txi[4] = {0.0, 0.0, 0.0, 0.0}, tyi[4] = {0.0, 0.0, 0.0, 0.0}, myi = 0.0, mxi = 0.0;
        Tw(gx, gy, td);
        if (a.k.extrap) {
            if (atL || atR) {  // the x wall's inward node
                const int xi = atL ? gx + 1 : gx - 1;
                Tw(xi, gy, txi);
#pragma unroll
                for (int q = 2; q < 9; q++)
                    if (ey(q) != 0) myi += pop_get<PR>(a.fsrc, g, gy, xi, q, finv);
            }
            if (wyB || wyT) {  // the y wall's inward node
                const int yi = wyB ? gy + 1 : gy - 1;
                Tw(gx, yi, tyi);
#pragma unroll
                for (int q = 1; q < 9; q++)
                    if (ex(q) != 0) mxi += pop_get<PR>(a.fsrc, g, yi, gx, q, finv);
            }
        }
        apply_walls(a.w, a.k, atL, atR, wyB, wyT, fo, sc[0], sc[1], td, txi[0], txi[2], myi, tyi[1], tyi[3], mxi, f);
    }
    // moments and the trapezoidal displacement update
    double m1x = 0.0, m1y = 0.0, o1x = 0.0, o1y = 0.0;
#pragma unroll
    for (int q = 0; q < 9; q++) {
        m1x += ex(q) * f[q];
        m1y += ey(q) * f[q];
        o1x += ex(q) * fo[q];
        o1y += ey(q) * fo[q];
    }
    double sn[2];
    sig_n(sn);
    const size_t ox = u_at(g, 0, gy, gx), oy = u_at(g, 1, gy, gx);
    a.udst[ox] = a.usrc[ox] + a.k.ucoef * (m1x + o1x + 0.5 * (sn[0] + sc[0]));
    a.udst[oy] = a.usrc[oy] + a.k.ucoef * (m1y + o1y + 0.5 * (sn[1] + sc[1]));
    double fn[9];
    collide_node<TWO_RATES>(f, collide_rates(a.k.omega, a.k.omega_p), fn);
    pop_put_all<PR>(a.fdst, g, gy, gx, fn, a.k.fscale);
}

template <int PR, bool TWO_RATES>
__global__ __launch_bounds__(256) void pass_step_kernel(PassArgs pa) {
    const StepArgs& a = pa.s;
    const Geometry& g = a.g;
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (gx >= g.nx || gy >= g.ny) return;
    const size_t plane = (size_t)g.plane;
    auto sig_c = [&](int x, int y, double s[2]) {
        const size_t oo = (size_t)y * g.pitch + x;
        s[0] = pa.sig_c[oo];
        s[1] = pa.sig_c[plane + oo];
    };
    auto sig_n = [&](double s[2]) {
        const size_t oo = (size_t)gy * g.pitch + gx;
        s[0] = pa.sig[oo];
        s[1] = pa.sig[plane + oo];
    };
    auto Tw = [&](int x, int y, double t[4]) {
        const size_t oo = (size_t)y * g.pitch + x;
#pragma unroll
        for (int c = 0; c < 4; c++) t[c] = pa.Tw[(size_t)c * plane + oo];
    };
    node_update<PR, TWO_RATES>(a, gx, gy, sig_c, sig_n, Tw);
}

// ---- the wall blocks of the fused step ----------------------------------------------------
//
// The march stores nothing at the nodes on non-periodic sides; wall blocks
// update them in FP64 (node_update: the walls of Sect. 3.3 with T and sigma of
// u_n, first-order boundary differences), in the march's launch after its
// blocks (march_kernel's fused form, march_wall_batch_kernel).  A wall block takes a segment of
// kWallSeg nodes of one side (the rows 0 and ny - 1 of non-periodic y sides
// whole, the columns 0 and nx - 1 of non-periodic x sides between them): it
// computes T on the three node lines nearest the wall and sigma on the two
// nearest into LDS, then one thread per wall node updates it from those.

struct WallBand {
    double T[3][kWallSeg + 4][4];  // [distance from the wall][along, from start - 2][comp]
    double S[2][kWallSeg + 2][2];  // [distance][along, from start - 1][comp]
};

template <int PR, int MAT>
__device__ __forceinline__ void wall_segment(const StepArgs& a, int seg, WallBand& band) {
    const Geometry& g = a.g;
    const WallSegs ws = wall_segs(g);
    // side: 0 bottom row, 1 top row, 2 left column, 3 right column
    int side, start;
    if (seg < 2 * ws.nrow) {
        side = seg / ws.nrow;
        start = (seg % ws.nrow) * kWallSeg;
    } else {
        const int k = seg - 2 * ws.nrow;
        side = 2 + k / ws.ncol;
        start = (g.py ? 0 : 1) + (k % ws.ncol) * kWallSeg;
    }
    const bool rowside = side < 2;
    const int len = rowside ? g.nx : g.ny;                        // nodes along the wall
    const int per = rowside ? g.px : g.py;                        // periodic along it
    const int end = rowside ? g.nx : (g.py ? g.ny : g.ny - 1);    // wall nodes of this side: [.., end)
    // node (x, y) at along-wall index t and distance d from the wall
    auto node = [&](int t, int d, int* x, int* y) {
        if (rowside) { *x = t; *y = side == 0 ? d : g.ny - 1 - d; }
        else { *y = t; *x = side == 2 ? d : g.nx - 1 - d; }
    };
    auto along = [&](int t, bool* ok) {  // an along-wall index into the lattice, wrapped if periodic
        if (per) return wrap(t, len);
        *ok = *ok && t >= 0 && t < len;
        return t;
    };
    const InitLike b = init_like(a, 1);
    // T on the three nearest lines, from u_n
    for (int k = threadIdx.x; k < 3 * (kWallSeg + 4); k += blockDim.x) {
        const int d = k / (kWallSeg + 4), i = k % (kWallSeg + 4);
        bool ok = true;
        const int t = along(start - 2 + i, &ok);
        if (!ok) continue;
        int x, y;
        node(t, d, &x, &y);
        node_T<MAT>(b, x, y, band.T[d][i]);
    }
    __syncthreads();
    // band entries of a node (x, y) near the segment: its distance from the wall
    // and its along-wall index relative to the band's first (periodic: the
    // representative in range; band entries of the same node hold the same values)
    auto dist = [&](int x, int y) {
        return rowside ? (side == 0 ? y : g.ny - 1 - y) : (side == 2 ? x : g.nx - 1 - x);
    };
    auto rel = [&](int x, int y, int first) {
        const int i = (rowside ? x : y) - first;
        return per ? wrap(i, len) : i;
    };
    auto Tband = [&](int x, int y, double t[4]) {
        const int dd = dist(x, y), i = rel(x, y, start - 2);
#pragma unroll
        for (int c = 0; c < 4; c++) t[c] = band.T[dd][i][c];
    };
    // sigma on the two nearest lines, from that T
    for (int k = threadIdx.x; k < 2 * (kWallSeg + 2); k += blockDim.x) {
        const int d = k / (kWallSeg + 2), i = k % (kWallSeg + 2);
        bool ok = true;
        const int t = along(start - 1 + i, &ok);
        if (!ok) continue;
        int x, y;
        node(t, d, &x, &y);
        sigma_from(b, x, y, Tband, band.S[d][i]);
    }
    __syncthreads();
    // the wall nodes
    const int t = start + (int)threadIdx.x;
    if ((int)threadIdx.x >= kWallSeg || t >= end) return;
    int gx, gy;
    node(t, 0, &gx, &gy);
    auto Sband = [&](int x, int y, double s[2]) {
        const int dd = dist(x, y), i = rel(x, y, start - 1);
        s[0] = band.S[dd][i][0];
        s[1] = band.S[dd][i][1];
    };
    auto sig_n = [&](double s[2]) { Sband(gx, gy, s); };
    if (a.k.omega_p != a.k.omega) node_update<PR, true>(a, gx, gy, Sband, sig_n, Tband);
    else node_update<PR, false>(a, gx, gy, Sband, sig_n, Tband);
}

// LDS of a step block: the four waves' halo blocks, or a wall segment's band
template <int PR, int HR>
union StepLds {
    HaloOf<PR, HR> halo[4];
    WallBand band;
};

// The step of one lattice: one work item per wave.  FUSED (every lattice with
// a non-periodic side): the launch also carries the wall segments, its last
// nwall blocks, which update the nodes on those sides.  Both kinds of block
// read only level n.  Last,
// the wall blocks take the slots the march's final round leaves idle: first,
// they held every slot at the march's start (walls last: 8192^2 tension +0.7 %
// in FP32; 2048 x 128 +8 % in FP32 and FP64; 1024^2 +1 % and +4 %).  (The
// 16-bit formats' fused kernel spilled while wall_segment was a call, and
// ran 25 % slower; inlined, it fits 240 registers.)  Two waves per SIMD, but
// one in FP64:
// its loop needs about 306 registers, and at two waves (256 each) the 50
// spilled to scratch cost more than the halved occupancy (8192^2 tension:
// 26.9k MLUPS at two waves, 28.4k at one).
template <int PR, int MAT, int HR, int D, bool FUSED>
__global__ __launch_bounds__(256, PR == PREC_F64 ? 1 : 2) void march_kernel(StepArgs a, int nwall, int nstrip,
                                                                             int nchunk, int chunk) {
    using Lds = typename std::conditional<FUSED, StepLds<PR, HR>, HaloOf<PR, HR>[4]>::type;
    __shared__ Lds lds;
    const int nmarch = (int)gridDim.x - nwall;  // march blocks, then wall blocks
    if constexpr (FUSED) {
        if ((int)blockIdx.x >= nmarch) {
            const int seg = (int)blockIdx.x - nmarch;
            if (seg < wall_segs(a.g).total) {
                const StepArgs la = a;  // a local copy: the argument block itself stays unaddressed
                wall_segment<PR, MAT>(la, seg, lds.band);
            }
            return;
        }
    }
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int item = __builtin_amdgcn_readfirstlane(xcd_tile((int)blockIdx.x, nmarch) * 4 + wv);
    if (item >= nstrip * nchunk) return;
    if constexpr (FUSED) march_item<PR, MAT, HR, D>(a, lds.halo[wv], lane, item % nstrip, item / nstrip, chunk);
    else march_item<PR, MAT, HR, D>(a, lds[wv], lane, item % nstrip, item / nstrip, chunk);
}

// The step of a batch of lattices of one material in one launch.  Its first
// march_blocks blocks march, one work item per wave, on a grid the host sizes
// to cover the table's items (extra waves end at once); a wave finds its
// simulation by bisection over the entries' first items (they are in
// simulation order), and the blocks that carry items are dealt to the XCDs in
// contiguous runs, as in march_kernel, so that neighbouring strips share their
// halo lines in one L2.  The blocks after them take one wall segment each,
// found by bisection over the entries' first segments.  Both kinds read only
// level n.  A simulation's waves read only its own buffers, so its results do
// not depend on its company.  No wave takes a second item: nothing is carried
// from one item to the next.  Placed last, the wall blocks fill the slots the
// march's final round leaves idle.  On the serving mix (200 requests,
// 1000..4000 steps) against a march launch followed by a wall launch: batched
// FP32 34.1 against 29.5 GLUPS, FP64 21.1 against 20.2, FP16 42.1 against
// 39.0; open-loop p50 0.23 s against 0.37 s and p99 0.43 s against 0.69 s.
// (With the wall blocks ahead of the march the step ran 35 % longer: the march
// needs about one round of resident blocks, and the wall blocks' slots pushed
// it into a second.)
template <int PR, int MAT, int HR, int D>
__global__ __launch_bounds__(256, PR == PREC_F64 ? 1 : 2) void march_wall_batch_kernel(
    const BatchStep* __restrict__ step, int march_blocks) {
    __shared__ StepLds<PR, HR> lds;
    const int nsims = step->nsims;
    if ((int)blockIdx.x >= march_blocks) {
        const int seg = (int)blockIdx.x - march_blocks;
        if (seg >= step->nsegs) return;
        int lo = 0, hi = nsims - 1;  // the last entry whose first segment is at or before seg
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (step->e[mid].seg0 <= seg) lo = mid;
            else hi = mid - 1;
        }
        const BatchEntry& e = step->e[lo];
        if (!e.skip) wall_segment<PR, MAT>(e.a, seg - e.seg0, lds.band);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int nitems = step->nitems;
    const int used = (nitems + 3) / 4;  // blocks that carry items
    if ((int)blockIdx.x >= used) return;
    const int item = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, used) * 4 + wv);
    if (item >= nitems) return;
    int lo = 0, hi = nsims - 1;  // the last entry whose first item is at or before item
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (step->e[mid].item0 <= item) lo = mid;
        else hi = mid - 1;
    }
    const BatchEntry& e = step->e[lo];
    if (e.skip) return;
    const int local = item - e.item0;
    march_item<PR, MAT, HR, D>(e.a, lds.halo[wv], lane, local % e.nstrip, local / e.nstrip, e.chunk);
}

hipError_t launch_stress_pass(int material, const InitLike& b, double* T, hipStream_t st) {
    const dim3 grid((b.g.nx + 63) / 64, (b.g.ny + 3) / 4), block(256);
    switch (material) {
    case MAT_SVK: hipLaunchKernelGGL((stress_pass_kernel<MAT_SVK>), grid, block, 0, st, b, T); break;
    case MAT_NH: hipLaunchKernelGGL((stress_pass_kernel<MAT_NH>), grid, block, 0, st, b, T); break;
    default: hipLaunchKernelGGL((stress_pass_kernel<MAT_LIN>), grid, block, 0, st, b, T); break;
    }
    return hipGetLastError();
}

hipError_t launch_source_pass(const InitLike& b, const double* T, double* sig, hipStream_t st) {
    const dim3 grid((b.g.nx + 63) / 64, (b.g.ny + 3) / 4), block(256);
    hipLaunchKernelGGL(source_pass_kernel, grid, block, 0, st, b, T, sig);
    return hipGetLastError();
}

template <int PR>
static void pass_step_p(const PassArgs& a, hipStream_t st) {
    const dim3 grid((a.s.g.nx + 63) / 64, (a.s.g.ny + 3) / 4), block(256);
    if (a.s.k.omega_p != a.s.k.omega) hipLaunchKernelGGL((pass_step_kernel<PR, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((pass_step_kernel<PR, false>), grid, block, 0, st, a);
}

hipError_t launch_pass_step(int prec, const PassArgs& a, hipStream_t st) {
    switch (prec) {
    case PREC_F64: pass_step_p<PREC_F64>(a, st); break;
    case PREC_F32: pass_step_p<PREC_F32>(a, st); break;
    case PREC_F16: pass_step_p<PREC_F16>(a, st); break;
    default: pass_step_p<PREC_BF16>(a, st); break;
    }
    return hipGetLastError();
}

// Failure scan: every node of every listed lattice, both displacement components;
// a wave that sees a value that is not finite, or a |u| above the entry's growth
// limit, raises its lattice's flag with one lane's buffer store (a vector store:
// no scalar-cache writes; concurrent stores all write 1).
constexpr int kScanBlocks = 1024;

__global__ __launch_bounds__(256) void nanscan_kernel(const ScanEntry* __restrict__ tab, int n,
                                                      uint32_t* __restrict__ flags) {
    const int lane = threadIdx.x & 63;
    const uint32_t nthreads = gridDim.x * blockDim.x;
    for (int e = 0; e < n; e++) {
        const ScanEntry s = tab[e];
        const uint32_t nodes = (uint32_t)s.nx * (uint32_t)s.ny, nx = (uint32_t)s.nx;
        bool bad = false;
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nodes; i += nthreads) {
            const size_t o = (size_t)(i / nx) * 2 * (size_t)s.pitch + i % nx;  // row records
            const double ux = s.u[o], uy = s.u[o + (size_t)s.pitch];
            bad |= !isfinite(ux) || !isfinite(uy) || (s.limit2 > 0.0 && ux * ux + uy * uy > s.limit2);
        }
        const uint64_t any = __builtin_amdgcn_ballot_w64(bad);
        if (any && lane == (int)__builtin_ctzll(any))
            __builtin_amdgcn_raw_buffer_store_b32(1u, rsrc(flags + s.slot, 4), 0u, 0u, 0);
    }
}

hipError_t launch_nanscan(const ScanEntry* tab, int n, uint32_t* flags, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(nanscan_kernel, dim3(kScanBlocks), dim3(256), 0, st, tab, n, flags);
    return hipGetLastError();
}

// ---- launchers ---------------------------------------------------------------------------------

// Waves per launch of march_kernel to aim for, by population storage (on large
// FP32 and FP64 lattices march_rows aims for more).  Longer chunks prime fewer
// rows, more waves balance the tail.  On the 8192^2 lattice (before the
// large-lattice rule):
//   FP32 (2048 resident waves): 40960 waves (28-row chunks) gave 49.5k MLUPS;
//         8192 / 12288 / 16384 / 32768 gave 5 %, 4.5 %, 2 % and 0.3 % less,
//         49152 and 65536 the same;
//   FP64 (1024 resident waves): 32768 (34 rows) gave 29.5k; 16384 / 24576 / 49152
//         gave 0.6 %, 0.2 % and 0.6 % less;
//   FP16, BF16: 16384 (64 rows) gave 71.8k / 72.0k; 8192 / 12288 / 32768 gave
//         2 %, 3 % and 0.7 % less.
template <int PR>
constexpr long march_waves() {
    return PR == PREC_F32 ? 40960 : (PR == PREC_F64 ? 32768 : 16384);
}

// rows per chunk of march_kernel: a multiple of its iterations per loop trip
// minus the two priming rows, with about `target` work items in all
static int march_chunk(const Geometry& g, int nstrip, int L, long target) {
    long c = ((long)g.ny * nstrip + target - 1) / target;
    long m = (c + 2 + L - 1) / L;
    if (m < 1) m = 1;
    if (m * L - 2 > 190) m = (190 + 2) / L;
    return (int)(m * L - 2);
}

// Rows per chunk for one lattice: about march_waves<PR>() work items; for FP32
// and FP64, on lattices large enough for 65536 work items of 16 rows or more,
// 16 rows.  Short chunks started together keep neighbouring waves in step, so
// more halo gathers find their lines in the L2 (8192^2 FP32: 4.33 GB read per
// launch against 4.74 with 28 rows).  Measured (MLUPS): 8192^2, 16 rows
// against 28 and 34: FP32 51.2k against 50.4k, FP64 29.8k against 29.2k (10
// rows: 50.2k and 29.6k); 12288^2, 16 rows against 40: 50.2k against 49.3k
// and 29.6k against 28.9k.  On 4096^2 the 65536 items would be 4-row chunks:
// FP32 38.8k against 49.4k with its 10 rows, FP64 28.0k against 30.8k.  FP16
// and BF16 keep 64 rows (34: -0.4 %, 22: -1.7 %, 16: -2 %).
constexpr long kMarchWavesLarge = 65536;
constexpr int kMarchRowsLarge = 16;
template <int PR>
static int march_rows(const Geometry& g, int nstrip, int L) {
    if constexpr (PR == PREC_F32 || PR == PREC_F64) {
        // (a chunk is a whole number of loop trips less the two priming rows)
        if ((kMarchRowsLarge + 2) % L == 0 && march_chunk(g, nstrip, L, kMarchWavesLarge) >= kMarchRowsLarge)
            return kMarchRowsLarge;
    }
    return march_chunk(g, nstrip, L, march_waves<PR>());
}

template <int PR, int MAT, int HR, int D>
static void launch_march(const StepArgs& a, bool fused, hipStream_t st) {
    constexpr int L = (HR % D == 0) ? HR : (D % HR == 0 ? D : HR * D);
    const int nstrip = a.g.pitch / 64;
    const int chunk = march_rows<PR>(a.g, nstrip, L);
    const int nchunk = (a.g.ny + chunk - 1) / chunk;
    const int blocks = (nstrip * nchunk + 3) / 4;
    if (fused) {
        const int nwall = wall_segs(a.g).total;
        hipLaunchKernelGGL((march_kernel<PR, MAT, HR, D, true>), dim3(nwall + blocks), dim3(256), 0, st, a, nwall,
                           nstrip, nchunk, chunk);
        return;
    }
    hipLaunchKernelGGL((march_kernel<PR, MAT, HR, D, false>), dim3(blocks), dim3(256), 0, st, a, 0, nstrip,
                       nchunk, chunk);
}

// Whether one lattice's step carries wall blocks (march_kernel's fused form):
// every lattice with a non-periodic side.  Measured, back-to-back steps,
// against the march followed by a launch of the wall blocks alone: FP32 gains
// at every size (tension32 and shear128 1.8-1.9x, 2048 x 128 +49 %, 1024^2
// +19 %, 2048^2 +5 %, 4096^2 +3 %, 8192^2 +0.7 %), FP16 too (8192^2 +2.3 %,
// 2048^2 +8 %, 1024^2 +21 %), and FP64 (1024^2 +10 %; with 16-row chunks and
// the wall segment inlined, 2048^2 +4 %, 4096^2 +1.9 %, 8192^2 +0.5 %).
bool step_fused(int prec, const Geometry& g) {
    (void)prec;
    return wall_segs(g).total > 0;
}

// In a batch the other lattices supply the waves: chunks of 16 rows (or the
// whole height, if less).  A step of a batch lasts about one chunk's march, so
// shorter chunks end it sooner, at the price of the two rows that prime each
// chunk, and short chunks started together keep neighbouring waves in step.
// On the serving mix (200 requests, 1000..4000 steps) 16 rows against 34:
// batched FP32 29.6 against 28.3 GLUPS, FP64 20.3 against 19.2, FP16 39.0
// against 38.1, open-loop p50 0.37 s against 0.50 s and p99 0.69 s against
// 0.84 s; 22 rows fell between.  (Before the state moved to row records, 34
// rows had been the fastest: 64 -9 %, 22 even, 10 -9 %.)
void march_shape(const Geometry& g, int* nstrip, int* nchunk, int* chunk) {
    *nstrip = g.pitch / 64;
    const int m = std::min(3, (g.ny + 2 + 5) / 6);
    *chunk = 6 * m - 2;
    *nchunk = (g.ny + *chunk - 1) / *chunk;
}

template <int PR>
static void batch_step_p(int material, const BatchStep* step, int march_blocks, int wall_blocks, hipStream_t st) {
    // one launch: the march blocks, then the wall blocks
    const dim3 grid(march_blocks + wall_blocks), block(256);
    if (material == MAT_SVK)
        hipLaunchKernelGGL((march_wall_batch_kernel<PR, MAT_SVK, 6, 2>), grid, block, 0, st, step, march_blocks);
    else
        hipLaunchKernelGGL((march_wall_batch_kernel<PR, MAT_NH, 6, 2>), grid, block, 0, st, step, march_blocks);
}

hipError_t launch_batch_step(int prec, int material, const BatchStep* step, int march_blocks, int wall_blocks,
                             hipStream_t st) {
    switch (prec) {
    case PREC_F64: batch_step_p<PREC_F64>(material, step, march_blocks, wall_blocks, st); break;
    case PREC_F32: batch_step_p<PREC_F32>(material, step, march_blocks, wall_blocks, st); break;
    case PREC_F16: batch_step_p<PREC_F16>(material, step, march_blocks, wall_blocks, st); break;
    default: batch_step_p<PREC_BF16>(material, step, march_blocks, wall_blocks, st); break;
    }
    return hipGetLastError();
}

template <int PR>
static hipError_t step_p(int material, const StepArgs& a, bool fused, hipStream_t st) {
    // halo blocks of 6 rows, loads of 2 rows in flight: the fastest of the
    // shapes measured on the 8192^2 workload (halo blocks of 2 to 6 rows, 2 or 3
    // rows in flight), in FP32 and FP64
    switch (material) {
    case MAT_SVK: launch_march<PR, MAT_SVK, 6, 2>(a, fused, st); break;
    case MAT_NH: launch_march<PR, MAT_NH, 6, 2>(a, fused, st); break;
    default: launch_march<PR, MAT_LIN, 6, 2>(a, fused, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_step(int prec, int material, const StepArgs& a, bool fused, hipStream_t st) {
    switch (prec) {
    case PREC_F64: return step_p<PREC_F64>(material, a, fused, st);
    case PREC_F32: return step_p<PREC_F32>(material, a, fused, st);
    case PREC_F16: return step_p<PREC_F16>(material, a, fused, st);
    default: return step_p<PREC_BF16>(material, a, fused, st);
    }
}

// ---- plain copy: the reference kernel for hardware byte counters -------------------------------

__global__ __launch_bounds__(256) void copy_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                   size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const float v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
        dst[i] = v0;
        dst[i + stride] = v1;
        dst[i + 2 * stride] = v2;
        dst[i + 3 * stride] = v3;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_copy(void* dst, const void* src, size_t n4, hipStream_t st) {
    if (n4 == 0) return hipSuccess;
    size_t blocks = (n4 + 255) / 256;
    if (blocks > 256 * 32) blocks = 256 * 32;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<const float*>(src),
                       static_cast<float*>(dst), n4);
    return hipGetLastError();
}

hipError_t launch_init(int prec, const InitArgs& a, hipStream_t st) {
    const dim3 grid((a.b.g.nx + 63) / 64, (a.b.g.ny + 3) / 4), block(256);
    switch (prec) {
    case PREC_F64: hipLaunchKernelGGL((init_kernel<PREC_F64>), grid, block, 0, st, a); break;
    case PREC_F32: hipLaunchKernelGGL((init_kernel<PREC_F32>), grid, block, 0, st, a); break;
    case PREC_F16: hipLaunchKernelGGL((init_kernel<PREC_F16>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((init_kernel<PREC_BF16>), grid, block, 0, st, a); break;
    }
    return hipGetLastError();
}

template <int PR>
static hipError_t read_p(int material, const ReadArgs& a, hipStream_t st) {
    const dim3 grid((a.b.g.nx + 63) / 64, (a.b.g.ny + 3) / 4), block(256);
    switch (material) {
    case MAT_SVK: hipLaunchKernelGGL((read_kernel<PR, MAT_SVK>), grid, block, 0, st, a); break;
    case MAT_NH: hipLaunchKernelGGL((read_kernel<PR, MAT_NH>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((read_kernel<PR, MAT_LIN>), grid, block, 0, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_read(int prec, int material, const ReadArgs& a, hipStream_t st) {
    switch (prec) {
    case PREC_F64: return read_p<PREC_F64>(material, a, st);
    case PREC_F32: return read_p<PREC_F32>(material, a, st);
    case PREC_F16: return read_p<PREC_F16>(material, a, st);
    default: return read_p<PREC_BF16>(material, a, st);
    }
}

int diag_blocks(const Geometry& g) { return ((g.nx + 63) / 64) * ((g.ny + 3) / 4); }

template <int PR>
static hipError_t diag_p(int material, const ReadArgs& a, double* out, int64_t* watch, int64_t step,
                         hipStream_t st, int nblk) {
    switch (material) {
    case MAT_SVK: hipLaunchKernelGGL((diag_kernel<PR, MAT_SVK>), dim3(nblk), dim3(256), 0, st, a); break;
    case MAT_NH: hipLaunchKernelGGL((diag_kernel<PR, MAT_NH>), dim3(nblk), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((diag_kernel<PR, MAT_LIN>), dim3(nblk), dim3(256), 0, st, a); break;
    }
    hipLaunchKernelGGL(diag_reduce_kernel, dim3(1), dim3(256), 0, st, static_cast<const double*>(a.partial), nblk,
                       out, watch, step);
    return hipGetLastError();
}

static hipError_t diag_any(int prec, int material, const ReadArgs& a, double* out, int64_t* watch, int64_t step,
                           hipStream_t st, int nblk) {
    switch (prec) {
    case PREC_F64: return diag_p<PREC_F64>(material, a, out, watch, step, st, nblk);
    case PREC_F32: return diag_p<PREC_F32>(material, a, out, watch, step, st, nblk);
    case PREC_F16: return diag_p<PREC_F16>(material, a, out, watch, step, st, nblk);
    default: return diag_p<PREC_BF16>(material, a, out, watch, step, st, nblk);
    }
}

hipError_t launch_diag(int prec, int material, const ReadArgs& a, double* out, int64_t* watch, int64_t step,
                       hipStream_t st) {
    return diag_any(prec, material, a, out, watch, step, st, diag_blocks(a.b.g));
}

// ---- the diagnostics without a workspace: partial sums in a fixed device array ---------------------
//
// For callers that cannot allocate: the block partials and the result live in
// `scratch`, one copy per device for the life of the process, at most
// kScratchBlocks partials (the grid is capped at that many blocks, each taking
// several tiles), whatever the lattice.  Every call writes all the partials it
// reads, so nothing needs clearing; calls that overlap on one device race for
// the array.  Host code reaches the array only through the address
// hipGetSymbolAddress reports for the current device.

constexpr int kScratchBlocks = 1024;
constexpr int kScratchDoubles = (kScratchBlocks + 1) * 8;  // partials, then the 8-double result
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch[kMaxDevices] = {};

hipError_t launch_diag_noalloc(int prec, int material, ReadArgs a, double host_out[5], hipStream_t st) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    double* base;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch[dev]) {  // once per device, with that device current
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            g_scratch[dev] = static_cast<double*>(p);
        }
        base = g_scratch[dev];
    }
    const int nblk = std::min(diag_blocks(a.b.g), kScratchBlocks);
    if (nblk < 1 || (size_t)(nblk + 1) * 8 > (size_t)kScratchDoubles) return hipErrorInvalidValue;
    a.partial = base;
    double* out = base + (size_t)kScratchBlocks * 8;
    e = diag_any(prec, material, a, out, nullptr, 0, st, nblk);
    if (e == hipSuccess) e = hipMemcpyAsync(host_out, out, 5 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

}  // namespace mclbm
