// march_pattern: the memory pattern of march_kernel alone, without its
// arithmetic, halo or walls: the bandwidth ceiling that pattern sets.  A wave
// owns 64 aligned columns of a strip and marches a chunk of rows (two priming
// rows read, not stored), reading each node's population words and its two
// FP64 u values and writing them to the other buffer, with two rows of loads in
// flight, on the same block-to-XCD order as march_kernel.
//   Formats: FP32 (nine 32-bit populations), 16-bit (four 32-bit words and one
//   16-bit value, the FP16 and BF16 layout), FP64 (nine 64-bit populations), and
//   two wider forms of FP32 in row records: pairs (four 64-bit words of two
//   populations and one 32-bit value) and fours (two 128-bit words and one
//   32-bit value), the same 36 B per node in fewer, wider accesses.
//   Layouts: row records, [ny][component][pitch] (the state's layout), with a
//   buffer resource per lattice row of populations (as march_kernel) or one
//   per chunk, the row in the lane offset; and planar, [component][ny][pitch]
//   (one plane per component; three planes, or the four word planes, per
//   resource).
//   Chunks of 34 and 64 rows; two or one waves per SIMD (set with 64 or 96 KiB
//   of dynamic LDS per block).
// Prints one JSON line per case: the mean launch time over 20 launches and the
// rate in the kernel's compulsory bytes (104, 68, 176 B per node).
//
// Usage: march_pattern [n]   (an n x n lattice, default 8192)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                            \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            std::fprintf(stderr, "%s:%d %s\n", __FILE__, __LINE__, hipGetErrorString(e_)); \
            std::exit(1);                                                                \
        }                                                                                \
    } while (0)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
    const int q = nblk / 8, r = nblk % 8;
    const int xcd = bid % 8, k = bid / 8;
    return xcd * q + min(xcd, r) + k;
}

struct Args {
    const char* fs;
    char* fd;
    const char* us;
    char* ud;
    int nx, ny, pitch, nstrip, nchunk, chunk;
    long long plane;
};

// FMT 0: FP32, 1: 16-bit, 2: FP64, 3: FP32 in pairs, 4: FP32 in fours
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int FMT>
struct Fmt {
    static constexpr int NW = FMT == 1 ? 5 : (FMT == 3 ? 5 : (FMT == 4 ? 3 : 9));  // words per node
    static constexpr uint32_t node_bytes = (FMT == 0 || FMT >= 3) ? 36 : (FMT == 1 ? 18 : 72);
    static constexpr bool packed = FMT == 1 || FMT >= 3;
    __host__ __device__ static constexpr uint32_t es(int w) {
        return FMT == 0 ? 4 : (FMT == 1 ? (w < 4 ? 4 : 2) : (FMT == 3 ? (w < 4 ? 8 : 4) : (FMT == 4 ? (w < 2 ? 16 : 4) : 8)));
    }
};
template <int FMT>
struct Row {
    u32x4 w[Fmt<FMT>::NW];
    double u[2];
};

// MODE 0: planar; 1: row records, a resource per row; 2: row records, a resource per chunk
template <int FMT, int MODE>
__global__ __launch_bounds__(256) void probe(Args a) {
    static_assert(FMT < 3 || MODE != 0, "the wider FP32 forms are row records only");
    using F = Fmt<FMT>;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int item = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + wv);
    if (item >= a.nstrip * a.nchunk) return;
    const int strip = item % a.nstrip, chk = item / a.nstrip;
    const int x = strip * 64 + lane;
    const int yc = chk * a.chunk, ye = min(yc + a.chunk, a.ny);
    const int y0 = max(yc - 2, 0);
    const uint32_t P = (uint32_t)a.pitch, pl = (uint32_t)a.plane;
    constexpr bool RR = MODE != 0;
    const uint32_t rec = F::node_bytes * P;  // one lattice row's record of populations
    // MODE 2: the chunk's rows y0 .. ye - 1 through one resource per buffer
    const __amdgpu_buffer_rsrc_t cs = rsrc(a.fs + (size_t)y0 * rec, (uint32_t)(ye - y0) * rec),
                                 cd = rsrc(a.fd + (size_t)y0 * rec, (uint32_t)(ye - y0) * rec);
    // planar: resources of three planes (FP32, FP64) or of the word planes and the 16-bit plane
    __amdgpu_buffer_rsrc_t ps[3], pd[3];
    if (!RR) {
        if (FMT == 1) {
            ps[0] = ps[1] = rsrc(a.fs, 16 * pl);
            ps[2] = rsrc(a.fs + (size_t)16 * pl, 2 * pl);
            pd[0] = pd[1] = rsrc(a.fd, 16 * pl);
            pd[2] = rsrc(a.fd + (size_t)16 * pl, 2 * pl);
        } else {
            const uint32_t e = F::es(0);
            for (int k = 0; k < 3; k++) {
                ps[k] = rsrc(a.fs + (size_t)3 * k * pl * e, 3 * pl * e);
                pd[k] = rsrc(a.fd + (size_t)3 * k * pl * e, 3 * pl * e);
            }
        }
    }
    const __amdgpu_buffer_rsrc_t us = rsrc(a.us, 16 * pl), ud = rsrc(a.ud, 16 * pl);
    // word w of row r: the resource, the lane's offset and the wave's offset
    auto where = [&](const char* base, const __amdgpu_buffer_rsrc_t* pr, int r, int w, __amdgpu_buffer_rsrc_t& rs,
                     uint32_t& vo, uint32_t& so) {
        if (MODE == 2) {
            rs = base == a.fs ? cs : cd;
            vo = (uint32_t)(r - y0) * rec + (uint32_t)x * F::es(w);
            so = F::packed ? (uint32_t)w * F::es(0) * P : (uint32_t)w * F::es(w) * P;
        } else if (RR) {
            rs = rsrc(base + (size_t)r * rec, rec);
            vo = (uint32_t)x * F::es(w);
            so = F::packed ? (uint32_t)w * F::es(0) * P : (uint32_t)w * F::es(w) * P;
        } else if (FMT == 1) {
            rs = pr[w < 4 ? 0 : 2];
            vo = (uint32_t)(r * P + x) * F::es(w);
            so = w < 4 ? (uint32_t)w * pl * 4u : 0u;
        } else {
            rs = pr[w / 3];
            vo = (uint32_t)(r * P + x) * F::es(w);
            so = (uint32_t)(w % 3) * pl * F::es(w);
        }
    };
    // u: [ny][2][pitch] (row records) or [2][ny][pitch]
    auto uwhere = [&](int r, int c, uint32_t& vo, uint32_t& so) {
        vo = (uint32_t)((RR ? 2 * r : r) * P + x) * 8u;
        so = (uint32_t)c * (RR ? P : pl) * 8u;
    };
    auto load = [&](int r, Row<FMT>& R) {
#pragma unroll
        for (int w = 0; w < F::NW; w++) {
            __amdgpu_buffer_rsrc_t rs;
            uint32_t vo, so;
            where(a.fs, ps, r, w, rs, vo, so);
            if (F::es(w) == 16) R.w[w] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0));
            else if (F::es(w) == 8) { const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0); R.w[w].x = v.x; R.w[w].y = v.y; }
            else if (F::es(w) == 4) R.w[w].x = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0);
            else R.w[w].x = __builtin_amdgcn_raw_buffer_load_b16(rs, vo, so, 0);
        }
#pragma unroll
        for (int c = 0; c < 2; c++) {
            uint32_t vo, so;
            uwhere(r, c, vo, so);
            R.u[c] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(us, vo, so, 0));
        }
    };
    auto store = [&](int r, const Row<FMT>& R) {
#pragma unroll
        for (int w = 0; w < F::NW; w++) {
            __amdgpu_buffer_rsrc_t rs;
            uint32_t vo, so;
            where(a.fd, pd, r, w, rs, vo, so);
            if (F::es(w) == 16) __builtin_amdgcn_raw_buffer_store_b128(R.w[w], rs, vo, so, 2);
            else if (F::es(w) == 8) { u32x2 v; v.x = R.w[w].x; v.y = R.w[w].y; __builtin_amdgcn_raw_buffer_store_b64(v, rs, vo, so, 2); }
            else if (F::es(w) == 4) __builtin_amdgcn_raw_buffer_store_b32(R.w[w].x, rs, vo, so, 2);
            else __builtin_amdgcn_raw_buffer_store_b16((unsigned short)R.w[w].x, rs, vo, so, 2);
        }
#pragma unroll
        for (int c = 0; c < 2; c++) {
            uint32_t vo, so;
            uwhere(r, c, vo, so);
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, R.u[c]), ud, vo, so, 2);
        }
    };
    // two rows of loads in flight ahead of the row stored
    Row<FMT> A, B, C;
    int r = y0;
    load(r, A);
    if (r + 1 < ye) load(r + 1, B);
    for (; r < ye; r += 3) {
        if (r + 2 < ye) load(r + 2, C);
        if (r >= yc) store(r, A);
        if (r + 1 >= ye) break;
        if (r + 3 < ye) load(r + 3, A);
        if (r + 1 >= yc) store(r + 1, B);
        if (r + 2 >= ye) break;
        if (r + 4 < ye) load(r + 4, B);
        if (r + 2 >= yc) store(r + 2, C);
    }
}

template <int FMT, int MODE>
static void run(const char* name, char* f0, char* f1, char* u0, char* u1, int nx, int ny, hipEvent_t e0,
                hipEvent_t e1) {
    const int pitch = (nx + 63) / 64 * 64;
    const long long plane = (long long)ny * pitch;
    const double bpn = (FMT == 0 || FMT >= 3) ? 104 : (FMT == 1 ? 68 : 176);
    CK(hipFuncSetAttribute((const void*)probe<FMT, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 << 10));
    for (int chunk : {34, 64}) {
        for (int lds : {64 << 10, 96 << 10}) {
            Args a{f0, f1, u0, u1, nx, ny, pitch, pitch / 64, (ny + chunk - 1) / chunk, chunk, plane};
            const int items = a.nstrip * a.nchunk, blocks = (items + 3) / 4;
            // host check of the grid against the buffers: the last node any wave
            // touches lies in them, and every item has a wave
            const long long last = (long long)(ny - 1) * pitch + (pitch - 1);
            if (last >= plane || (long long)blocks * 4 < items) {
                std::fprintf(stderr, "bad grid\n");
                std::exit(1);
            }
            auto launch = [&](int k) {
                Args b = a;
                if (k & 1) {
                    b.fs = f1;
                    b.fd = f0;
                    b.us = u1;
                    b.ud = u0;
                }
                hipLaunchKernelGGL((probe<FMT, MODE>), dim3(blocks), dim3(256), lds, 0, b);
            };
            for (int k = 0; k < 4; k++) launch(k);
            CK(hipDeviceSynchronize());
            const int reps = 20;
            CK(hipEventRecord(e0));
            for (int k = 0; k < reps; k++) launch(k);
            CK(hipEventRecord(e1));
            CK(hipEventSynchronize(e1));
            CK(hipGetLastError());
            float ms = 0;
            CK(hipEventElapsedTime(&ms, e0, e1));
            const double per = ms / reps;
            std::printf("{\"format\": \"%s\", \"layout\": \"%s\", \"chunk\": %d, \"waves_per_simd\": %d, "
                        "\"ms\": %.4f, \"TBps_compulsory\": %.3f}\n",
                        name, MODE == 2 ? "row_records_chunk" : (MODE == 1 ? "row_records" : "planar"), chunk, lds == (64 << 10) ? 2 : 1, per,
                        bpn * nx * ny / (per * 1e-3) / 1e12);
            std::fflush(stdout);
        }
    }
}

int main(int argc, char** argv) {
    const int n = argc > 1 ? std::atoi(argv[1]) : 8192;
    const int nx = n, ny = n, pitch = (nx + 63) / 64 * 64;
    const long long plane = (long long)ny * pitch;
    // 32-bit ranges: the planar layout's three FP64 planes, and a u buffer
    if (plane * 24 >= (1ll << 32) || plane * 16 >= (1ll << 32)) {
        std::fprintf(stderr, "lattice too large for 32-bit offsets\n");
        return 1;
    }
    const size_t fbytes = (size_t)plane * 72, ubytes = (size_t)plane * 16;
    char *f0, *f1, *u0, *u1;
    CK(hipMalloc(&f0, fbytes));
    CK(hipMalloc(&f1, fbytes));
    CK(hipMalloc(&u0, ubytes));
    CK(hipMalloc(&u1, ubytes));
    CK(hipMemset(f0, 1, fbytes));
    CK(hipMemset(f1, 1, fbytes));
    CK(hipMemset(u0, 0, ubytes));
    CK(hipMemset(u1, 0, ubytes));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    run<0, 1>("fp32", f0, f1, u0, u1, nx, ny, e0, e1);
    run<0, 2>("fp32", f0, f1, u0, u1, nx, ny, e0, e1);
    run<0, 0>("fp32", f0, f1, u0, u1, nx, ny, e0, e1);
    run<3, 1>("fp32_pairs", f0, f1, u0, u1, nx, ny, e0, e1);
    run<3, 2>("fp32_pairs", f0, f1, u0, u1, nx, ny, e0, e1);
    run<4, 1>("fp32_quads", f0, f1, u0, u1, nx, ny, e0, e1);
    run<4, 2>("fp32_quads", f0, f1, u0, u1, nx, ny, e0, e1);
    run<1, 1>("16bit", f0, f1, u0, u1, nx, ny, e0, e1);
    run<1, 2>("16bit", f0, f1, u0, u1, nx, ny, e0, e1);
    run<1, 0>("16bit", f0, f1, u0, u1, nx, ny, e0, e1);
    run<2, 1>("fp64", f0, f1, u0, u1, nx, ny, e0, e1);
    run<2, 2>("fp64", f0, f1, u0, u1, nx, ny, e0, e1);
    run<2, 0>("fp64", f0, f1, u0, u1, nx, ny, e0, e1);
    return 0;
}
