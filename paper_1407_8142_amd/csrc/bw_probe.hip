// bw_probe: streaming probes of the achievable HBM bandwidth, and the
// known-size kernels that calibrate rocprofv3 FETCH_SIZE / WRITE_SIZE.
//   copy_u4     grid-stride copy with 16-byte loads and stores
//   copy_tile   one 16 KiB tile per block, four 16-byte loads per thread
//               issued together, then the stores: the level pass's access
//               pattern without its work
//   read_tile   the same loads, no stores (a sum per block, written once)
// Each prints one JSON line with bytes per launch and GB/s.
//   bw_probe [MiB per buffer, default 1024] [iterations, default 20]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

__global__ __launch_bounds__(256) void copy_u4(const uint4 *__restrict__ a, uint4 *__restrict__ b, size_t n) {
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// n16 = number of 16-byte words, a multiple of 1024 (whole tiles).
__global__ __launch_bounds__(256) void copy_tile(const uint4 *__restrict__ a, uint4 *__restrict__ b) {
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
    uint4 q[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) q[r] = a[base + 256 * r];
#pragma unroll
    for (int r = 0; r < 4; ++r) b[base + 256 * r] = q[r];
}

__global__ __launch_bounds__(256) void read_tile(const uint4 *__restrict__ a, unsigned *__restrict__ sink) {
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
    uint4 q[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) q[r] = a[base + 256 * r];
    unsigned x = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) x ^= q[r].x ^ q[r].y ^ q[r].z ^ q[r].w;
    if (x == 0x9E3779B9u) sink[blockIdx.x & 1023] = x;  // keeps the loads; practically never taken
}

#define CHECK(x)                                                              \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));    \
            return 1;                                                         \
        }                                                                     \
    } while (0)

int main(int argc, char **argv) {
    size_t mib = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1024;
    int iters = argc > 2 ? atoi(argv[2]) : 20;
    if (mib == 0 || iters <= 0) return 2;
    size_t bytes = mib << 20, n = bytes / sizeof(uint4);  // a multiple of 1024 16-byte words
    uint4 *a = nullptr, *b = nullptr;
    unsigned *sink = nullptr;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    CHECK(hipMalloc(&sink, 4096));
    CHECK(hipMemset(a, 1, bytes));
    CHECK(hipMemset(b, 0, bytes));
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const unsigned grid = (unsigned)(cus * 16), tiles = (unsigned)(n / 1024);
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int kind = 0; kind < 3; ++kind) {
        auto launch = [&]() {
            if (kind == 0) copy_u4<<<grid, 256>>>(a, b, n);
            else if (kind == 1) copy_tile<<<tiles, 256>>>(a, b);
            else read_tile<<<tiles, 256>>>(a, sink);
        };
        for (int w = 0; w < 5; ++w) launch();
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(e0, 0));
        for (int i = 0; i < iters; ++i) launch();
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipGetLastError());
        float ms = 0;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        const size_t wr = kind == 2 ? 0 : bytes;
        const double gbs = (double)(bytes + wr) * iters / (ms / 1e3) / 1e9;
        const char *name = kind == 0 ? "copy_u4" : (kind == 1 ? "copy_tile" : "read_tile");
        printf("{\"probe\": \"%s\", \"bytes_read_per_launch\": %zu, \"bytes_written_per_launch\": %zu, "
               "\"avg_launch_ms\": %.5f, \"GBps\": %.1f, \"cus\": %d}\n",
               name, bytes, wr, ms / iters, gbs, cus);
    }
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(sink));
    return 0;
}
