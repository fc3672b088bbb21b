// march_pattern: the memory pattern of march_kernel alone, without its
// arithmetic, halo or walls: the bandwidth ceiling that pattern sets.  A wave
// owns 64 aligned columns of a strip and marches a chunk of rows (two priming
// rows read, not stored), reading each node's population words and its two
// FP64 u values and writing them to the other buffer, with two rows of loads in
// flight, on the same block-to-XCD order as march_kernel.  Formats: FP32 (9 x
// 32-bit planes), 16-bit (4 x 32-bit word planes + 1 x 16-bit plane, the FP16
// and BF16 layout), FP64 (9 x 64-bit planes); chunks of 34 and 64 rows; two or
// one waves per SIMD (set with 64 or 96 KiB of dynamic LDS per block).  Prints
// one JSON line per case: the mean launch time over 20 launches and the rate in
// the kernel's compulsory bytes (104, 68, 176 B per node).
//
// Usage: march_pattern [n]   (an n x n lattice, default 8192)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

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
    const double* us;
    double* ud;
    int nx, ny, pitch, nstrip, nchunk, chunk;
    long long plane;
};

template <int FMT>
struct Row {
    static constexpr int NW = FMT == 0 ? 9 : (FMT == 1 ? 5 : 9);
    uint64_t w[NW];
    double u[2];
};

template <int FMT>
__global__ __launch_bounds__(256) void probe(Args a) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int item = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * 4 + wv);
    if (item >= a.nstrip * a.nchunk) return;
    const int strip = item % a.nstrip, chk = item / a.nstrip;
    const int x = strip * 64 + lane;
    const int yc = chk * a.chunk, ye = min(yc + a.chunk, a.ny);
    const int y0 = max(yc - 2, 0);
    const uint32_t pl = (uint32_t)a.plane;
    // resources: three planes each (FP32, FP64), or four word planes + one 16-bit plane
    const uint32_t es = FMT == 2 ? 8u : 4u;
    __amdgpu_buffer_rsrc_t s0, s1, s2, d0, d1, d2;
    if (FMT == 1) {
        s0 = rsrc(a.fs, 4 * pl * 4);
        s1 = rsrc(a.fs + (size_t)4 * pl * 4, pl * 2);
        s2 = s1;
        d0 = rsrc(a.fd, 4 * pl * 4);
        d1 = rsrc(a.fd + (size_t)4 * pl * 4, pl * 2);
        d2 = d1;
    } else {
        s0 = rsrc(a.fs, 3 * pl * es);
        s1 = rsrc(a.fs + (size_t)3 * pl * es, 3 * pl * es);
        s2 = rsrc(a.fs + (size_t)6 * pl * es, 3 * pl * es);
        d0 = rsrc(a.fd, 3 * pl * es);
        d1 = rsrc(a.fd + (size_t)3 * pl * es, 3 * pl * es);
        d2 = rsrc(a.fd + (size_t)6 * pl * es, 3 * pl * es);
    }
    const __amdgpu_buffer_rsrc_t us = rsrc(a.us, 2 * pl * 8), ud = rsrc(a.ud, 2 * pl * 8);
    auto load = [&](int r, Row<FMT>& R) {
        const uint32_t node = (uint32_t)(r * a.pitch + x);
        if constexpr (FMT == 1) {
#pragma unroll
            for (int w = 0; w < 4; w++) R.w[w] = __builtin_amdgcn_raw_buffer_load_b32(s0, node * 4u, (uint32_t)w * pl * 4u, 0);
            R.w[4] = __builtin_amdgcn_raw_buffer_load_b16(s1, node * 2u, 0u, 0);
        } else if constexpr (FMT == 0) {
#pragma unroll
            for (int q = 0; q < 9; q++)
                R.w[q] = __builtin_amdgcn_raw_buffer_load_b32(q < 3 ? s0 : (q < 6 ? s1 : s2), node * 4u,
                                                              (uint32_t)(q % 3) * pl * 4u, 0);
        } else {
#pragma unroll
            for (int q = 0; q < 9; q++)
                R.w[q] = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(
                                                          q < 3 ? s0 : (q < 6 ? s1 : s2), node * 8u,
                                                          (uint32_t)(q % 3) * pl * 8u, 0));
        }
        R.u[0] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(us, node * 8u, 0u, 0));
        R.u[1] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(us, node * 8u, pl * 8u, 0));
    };
    auto store = [&](int r, const Row<FMT>& R) {
        const uint32_t node = (uint32_t)(r * a.pitch + x);
        if constexpr (FMT == 1) {
#pragma unroll
            for (int w = 0; w < 4; w++)
                __builtin_amdgcn_raw_buffer_store_b32((uint32_t)R.w[w], d0, node * 4u, (uint32_t)w * pl * 4u, 2);
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)R.w[4], d1, node * 2u, 0u, 2);
        } else if constexpr (FMT == 0) {
#pragma unroll
            for (int q = 0; q < 9; q++)
                __builtin_amdgcn_raw_buffer_store_b32((uint32_t)R.w[q], q < 3 ? d0 : (q < 6 ? d1 : d2), node * 4u,
                                                      (uint32_t)(q % 3) * pl * 4u, 2);
        } else {
#pragma unroll
            for (int q = 0; q < 9; q++)
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, R.w[q]),
                                                      q < 3 ? d0 : (q < 6 ? d1 : d2), node * 8u,
                                                      (uint32_t)(q % 3) * pl * 8u, 2);
        }
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, R.u[0]), ud, node * 8u, 0u, 2);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, R.u[1]), ud, node * 8u, pl * 8u, 2);
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

int main(int argc, char** argv) {
    const int n = argc > 1 ? std::atoi(argv[1]) : 8192;
    const int nx = n, ny = n, pitch = (nx + 63) / 64 * 64;
    const long long plane = (long long)ny * pitch;
    if (plane * 9 * 8 / 3 >= (1ll << 32) || plane * 16 >= (1ll << 32)) {
        std::fprintf(stderr, "lattice too large for 32-bit offsets\n");
        return 1;
    }
    const size_t fbytes = (size_t)plane * 9 * 8, ubytes = (size_t)plane * 2 * 8;
    char *f0, *f1;
    double *u0, *u1;
    CK(hipMalloc(&f0, fbytes));
    CK(hipMalloc(&f1, fbytes));
    CK(hipMalloc(&u0, ubytes));
    CK(hipMalloc(&u1, ubytes));
    CK(hipMemset(f0, 1, fbytes));
    CK(hipMemset(u0, 0, ubytes));
    CK(hipFuncSetAttribute((const void*)probe<0>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 << 10));
    CK(hipFuncSetAttribute((const void*)probe<1>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 << 10));
    CK(hipFuncSetAttribute((const void*)probe<2>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 << 10));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    const int fmts[3] = {0, 1, 2};
    const double bpn[3] = {104, 68, 176};
    const char* names[3] = {"fp32", "16bit", "fp64"};
    for (int fi = 0; fi < 3; fi++) {
        const int fmt = fmts[fi];
        for (int chunk : {34, 64}) {
            for (int lds : {64 << 10, 96 << 10}) {
                Args a{f0, f1, u0, u1, nx, ny, pitch, pitch / 64, (ny + chunk - 1) / chunk, chunk, plane};
                const int items = a.nstrip * a.nchunk, blocks = (items + 3) / 4;
                // host check of the grid against the buffers: the last node any wave touches
                const long long last = (long long)(ny - 1) * pitch + (pitch - 1);
                if (last >= plane || (long long)blocks * 4 < items) {
                    std::fprintf(stderr, "bad grid\n");
                    return 1;
                }
                auto launch = [&](int k) {
                    Args b = a;
                    if (k & 1) {
                        b.fs = f1;
                        b.fd = f0;
                        b.us = u1;
                        b.ud = u0;
                    }
                    if (fmt == 0) hipLaunchKernelGGL(probe<0>, dim3(blocks), dim3(256), lds, 0, b);
                    else if (fmt == 1) hipLaunchKernelGGL(probe<1>, dim3(blocks), dim3(256), lds, 0, b);
                    else hipLaunchKernelGGL(probe<2>, dim3(blocks), dim3(256), lds, 0, b);
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
                std::printf("{\"format\": \"%s\", \"chunk\": %d, \"waves_per_simd\": %d, \"ms\": %.4f, "
                            "\"TBps_compulsory\": %.3f}\n",
                            names[fi], chunk, lds == (64 << 10) ? 2 : 1, per, bpn[fi] * nx * ny / (per * 1e-3) / 1e12);
                std::fflush(stdout);
            }
        }
    }
    return 0;
}
