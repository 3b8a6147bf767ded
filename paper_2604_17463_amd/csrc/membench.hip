// Memory-system probe for the roofline of the stream-collide kernel (gfx950).
//
// Times plain device copies and the stream-collide's own access pattern with
// the collision removed: every thread reads the 19 population planes of one
// cell and writes them to the 19 planes of the other buffer, with plain or
// streaming (non-temporal) stores.  The result is the read+write bandwidth
// the HBM system delivers to such a pattern, the practical ceiling for a
// kernel that must read and write every population once.
//
//   paper_2604_17463_amd/membench [nx ny nz]     (default 256 256 128, FP32)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                      \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

typedef float f4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void copy_vec4(const f4 *__restrict__ a, f4 *__restrict__ b, size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
        const f4 v = a[i];
        if (NT)
            __builtin_nontemporal_store(v, b + i);
        else
            b[i] = v;
    }
}

template <bool NT>
__global__ void copy_planes(const float *__restrict__ a, float *__restrict__ b, size_t plane, size_t n) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) v[q] = a[q * plane + i];
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        if (NT)
            __builtin_nontemporal_store(v[q], b + q * plane + i);
        else
            b[q * plane + i] = v[q];
    }
}

// The same with 2-byte elements (the FP16/BF16 deviation storage): one cell
// per lane (2 B per access) or two neighbouring cells per lane (4 B).
template <typename T, bool NT>
__global__ void copy_planes_t(const T *__restrict__ a, T *__restrict__ b, size_t plane, size_t n) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    T v[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) v[q] = a[q * plane + i];
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        if (NT)
            __builtin_nontemporal_store(v[q], b + q * plane + i);
        else
            b[q * plane + i] = v[q];
    }
}

int main(int argc, char **argv) {
    size_t nx = 256, ny = 256, nz = 128;
    if (argc == 4) {
        nx = std::strtoull(argv[1], nullptr, 10);
        ny = std::strtoull(argv[2], nullptr, 10);
        nz = std::strtoull(argv[3], nullptr, 10);
    }
    const size_t n = nx * ny * nz, plane = n, total = 19 * plane;
    if (n == 0 || total * sizeof(float) > (size_t)64 << 30) {
        std::fprintf(stderr, "box size out of range\n");
        return 2;
    }
    float *a = nullptr, *b = nullptr;
    CK(hipMalloc(&a, total * sizeof(float)));
    CK(hipMalloc(&b, total * sizeof(float)));
    CK(hipMemset(a, 0, total * sizeof(float)));
    CK(hipMemset(b, 0, total * sizeof(float)));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    const double bytes = 2.0 * total * sizeof(float);
    auto run = [&](const char *name, auto launch) {
        for (int w = 0; w < 3; ++w) launch();
        CK(hipGetLastError());
        CK(hipDeviceSynchronize());
        float best = 1e30f;
        for (int r = 0; r < 5; ++r) {
            CK(hipEventRecord(e0));
            for (int k = 0; k < 20; ++k) launch();
            CK(hipEventRecord(e1));
            CK(hipEventSynchronize(e1));
            float ms = 0;
            CK(hipEventElapsedTime(&ms, e0, e1));
            if (ms / 20 < best) best = ms / 20;
        }
        std::printf("%-34s %9.1f us %8.1f GB/s\n", name, best * 1e3, bytes / (best * 1e-3) / 1e9);
        std::fflush(stdout);
    };
    std::printf("box %zux%zux%zu, 19 FP32 planes, %.1f MB read + %.1f MB written per pass\n", nx, ny, nz,
                total * 4e-6, total * 4e-6);
    const size_t n4 = total / 4;
    run("copy, 16 B per lane, 1024 x 256", [&] { copy_vec4<false><<<1024, 256>>>((const f4 *)a, (f4 *)b, n4); });
    run("copy, 16 B per lane, streaming", [&] { copy_vec4<true><<<1024, 256>>>((const f4 *)a, (f4 *)b, n4); });
    const unsigned g = (unsigned)((n + 255) / 256);
    run("19-plane read/write, plain", [&] { copy_planes<false><<<g, 256>>>(a, b, plane, n); });
    run("19-plane read/write, streaming", [&] { copy_planes<true><<<g, 256>>>(a, b, plane, n); });
    // 2-byte planes over the same cells: half the bytes per pass
    const double bytes2 = bytes / 2;
    auto run2 = [&](const char *name, auto launch) {
        for (int w = 0; w < 3; ++w) launch();
        CK(hipGetLastError());
        CK(hipDeviceSynchronize());
        float best = 1e30f;
        for (int r = 0; r < 5; ++r) {
            CK(hipEventRecord(e0));
            for (int k = 0; k < 20; ++k) launch();
            CK(hipEventRecord(e1));
            CK(hipEventSynchronize(e1));
            float ms = 0;
            CK(hipEventElapsedTime(&ms, e0, e1));
            if (ms / 20 < best) best = ms / 20;
        }
        std::printf("%-34s %9.1f us %8.1f GB/s\n", name, best * 1e3, bytes2 / (best * 1e-3) / 1e9);
        std::fflush(stdout);
    };
    const unsigned g2 = (unsigned)((n / 2 + 255) / 256);
    run2("2-byte planes, 2 B per lane", [&] {
        copy_planes_t<unsigned short, false><<<g, 256>>>((const unsigned short *)a, (unsigned short *)b, plane, n);
    });
    run2("2-byte planes, 2 B per lane, NT", [&] {
        copy_planes_t<unsigned short, true><<<g, 256>>>((const unsigned short *)a, (unsigned short *)b, plane, n);
    });
    run2("2-byte planes, 4 B per lane", [&] {
        copy_planes_t<unsigned, false><<<g2, 256>>>((const unsigned *)a, (unsigned *)b, plane / 2, n / 2);
    });
    run2("2-byte planes, 4 B per lane, NT", [&] {
        copy_planes_t<unsigned, true><<<g2, 256>>>((const unsigned *)a, (unsigned *)b, plane / 2, n / 2);
    });
    CK(hipFree(a));
    CK(hipFree(b));
    return 0;
}
