// bw_probe: streaming copy with 16-byte loads and stores.  Reports the
// achievable HBM copy bandwidth (read + write bytes / time) and serves as
// the known-size kernel that calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE.
//   bw_probe [MiB per buffer, default 1024] [iterations, default 20]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

__global__ __launch_bounds__(256) void copy_u4(const uint4 *__restrict__ a, uint4 *__restrict__ b, size_t n) {
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
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
    size_t bytes = mib << 20, n = bytes / sizeof(uint4);
    uint4 *a = nullptr, *b = nullptr;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    CHECK(hipMemset(a, 1, bytes));
    CHECK(hipMemset(b, 0, bytes));
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    unsigned grid = (unsigned)(cus * 16);
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int w = 0; w < 3; ++w) copy_u4<<<grid, 256>>>(a, b, n);
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0, 0));
    for (int i = 0; i < iters; ++i) copy_u4<<<grid, 256>>>(a, b, n);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    double gbs = 2.0 * (double)bytes * iters / (ms / 1e3) / 1e9;
    printf("{\"probe\": \"copy_u4\", \"bytes_read_per_launch\": %zu, \"bytes_written_per_launch\": %zu, "
           "\"avg_launch_ms\": %.5f, \"copy_GBps\": %.1f, \"cus\": %d}\n",
           bytes, bytes, ms / iters, gbs, cus);
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    return 0;
}
