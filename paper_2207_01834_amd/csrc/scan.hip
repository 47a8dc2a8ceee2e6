// Device-wide exclusive prefix sum of uint32 values (the parallel prefix sum
// the paper's construction and batch gathers rely on, Appendix C).
// Three passes: per-workgroup totals, a scan of the totals by one workgroup,
// then per-workgroup scans offset by their total's prefix.
#include "scan.hpp"
#include "wave.hpp"

namespace pg {

namespace {

constexpr int kNT = 256;
constexpr int kItems = 16;
constexpr int kTile = kNT * kItems;

__global__ void __launch_bounds__(kNT)
tile_sum_kernel(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ sums) {
    __shared__ uint32_t red[kNT / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t s = 0;
    for (int i = 0; i < kItems; i++) {
        const int64_t e = base + (int64_t)i * kNT + threadIdx.x;
        if (e < n) s += in[e];
    }
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kNT / kWave; w++) t += red[w];
        sums[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kNT)
scan_sums_kernel(uint32_t* __restrict__ sums, int64_t count, uint32_t* __restrict__ total) {
    __shared__ uint32_t lds[kNT / kWave + 1];
    uint32_t run = 0;
    for (int64_t b = 0; b < count; b += kNT) {
        const int64_t e = b + threadIdx.x;
        const uint32_t v = e < count ? sums[e] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kNT>(v, lds, &tot);
        if (e < count) sums[e] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0 && total) *total = run;
}

__global__ void __launch_bounds__(kNT)
tile_scan_kernel(const uint32_t* __restrict__ in, int64_t n, const uint32_t* __restrict__ sums,
                 uint32_t* __restrict__ out) {
    __shared__ uint32_t lds[kNT / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t run = sums[blockIdx.x];
    for (int i = 0; i < kItems; i++) {
        const int64_t e = base + (int64_t)i * kNT + threadIdx.x;
        const uint32_t v = e < n ? in[e] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kNT>(v, lds, &tot);
        if (e < n) out[e] = run + ex;
        run += tot;
    }
}

}  // namespace

pg_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                             hipStream_t s) {
    if (n <= 0) return PG_OK;
    const int64_t tiles = (n + kTile - 1) / kTile;
    DevBuf sums(s);
    PG_TRY(sums.alloc(sizeof(uint32_t) * tiles));
    hipLaunchKernelGGL(tile_sum_kernel, dim3((unsigned)tiles), dim3(kNT), 0, s, in, n,
                       sums.as<uint32_t>());
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kNT), 0, s, sums.as<uint32_t>(), tiles,
                       total);
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL(tile_scan_kernel, dim3((unsigned)tiles), dim3(kNT), 0, s, in, n,
                       sums.as<uint32_t>(), out);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

}  // namespace pg
