// Device-wide exclusive prefix sums (the parallel prefix sum
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

// IT: input type, AT: sum type.
template <typename IT, typename AT>
__global__ void __launch_bounds__(kNT)
tile_sum_kernel(const IT* __restrict__ in, int64_t n, AT* __restrict__ sums) {
    __shared__ AT red[kNT / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    AT s = 0;
    for (int i = 0; i < kItems; i++) {
        const int64_t e = base + (int64_t)i * kNT + threadIdx.x;
        if (e < n) s += (AT)in[e];
    }
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        AT t = 0;
        for (int w = 0; w < kNT / kWave; w++) t += red[w];
        sums[blockIdx.x] = t;
    }
}

template <typename AT>
__global__ void __launch_bounds__(kNT)
scan_sums_kernel(AT* __restrict__ sums, int64_t count, AT* __restrict__ total) {
    __shared__ AT lds[kNT / kWave + 1];
    AT run = 0;
    for (int64_t b = 0; b < count; b += kNT) {
        const int64_t e = b + threadIdx.x;
        const AT v = e < count ? sums[e] : AT(0);
        AT tot;
        const AT ex = block_excl_scan<kNT>(v, lds, &tot);
        if (e < count) sums[e] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0 && total) *total = run;
}

template <typename IT, typename AT>
__global__ void __launch_bounds__(kNT)
tile_scan_kernel(const IT* __restrict__ in, int64_t n, const AT* __restrict__ sums,
                 AT* __restrict__ out) {
    __shared__ AT lds[kNT / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    AT run = sums[blockIdx.x];
    for (int i = 0; i < kItems; i++) {
        const int64_t e = base + (int64_t)i * kNT + threadIdx.x;
        const AT v = e < n ? (AT)in[e] : AT(0);
        AT tot;
        const AT ex = block_excl_scan<kNT>(v, lds, &tot);
        if (e < n) out[e] = run + ex;
        run += tot;
    }
}

// sums: scan_partials(n) entries of workspace.
template <typename IT, typename AT>
pg_status exclusive_scan_ws(const IT* in, AT* out, int64_t n, AT* total, AT* sums, hipStream_t s) {
    if (n <= 0) return PG_OK;
    const int64_t tiles = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL((tile_sum_kernel<IT, AT>), dim3((unsigned)tiles), dim3(kNT), 0, s, in, n, sums);
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL((scan_sums_kernel<AT>), dim3(1), dim3(kNT), 0, s, sums, tiles, total);
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL((tile_scan_kernel<IT, AT>), dim3((unsigned)tiles), dim3(kNT), 0, s, in, n, sums,
                       out);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

template <typename IT, typename AT>
pg_status exclusive_scan(const IT* in, AT* out, int64_t n, AT* total, hipStream_t s) {
    if (n <= 0) return PG_OK;
    DevBuf sums(s);
    PG_TRY(sums.alloc(sizeof(AT) * scan_partials(n)));
    return exclusive_scan_ws<IT, AT>(in, out, n, total, sums.as<AT>(), s);
}

// The same three passes over a count read on the device, n = mul * *cnt +
// add, with grids sized for a bound on it: each workgroup takes tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...  The total is written whatever n
// (0 for an empty input), to *total and, with at_end, to out[n].
struct DevCount {
    const uint32_t* cnt;
    uint32_t mul, add;
    __device__ inline int64_t get() const { return (int64_t)mul * (int64_t)*cnt + add; }
};

template <typename IT, typename AT>
__global__ void __launch_bounds__(kNT)
tile_sum_dev_kernel(const IT* __restrict__ in, DevCount dc, AT* __restrict__ sums) {
    __shared__ AT red[kNT / kWave];
    const int64_t n = dc.get();
    const int64_t tiles = (n + kTile - 1) / kTile;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t base = t * kTile;
        AT s = 0;
        for (int i = 0; i < kItems; i++) {
            const int64_t e = base + (int64_t)i * kNT + threadIdx.x;
            if (e < n) s += (AT)in[e];
        }
        s = wave_sum(s);
        __syncthreads();  // the previous tile's totals are read
        if (lane_id() == 0) red[threadIdx.x / kWave] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            AT u = 0;
            for (int w = 0; w < kNT / kWave; w++) u += red[w];
            sums[t] = u;
        }
    }
}

template <typename AT>
__global__ void __launch_bounds__(kNT)
scan_sums_dev_kernel(AT* __restrict__ sums, DevCount dc, AT* __restrict__ total, AT* __restrict__ out,
                     int at_end) {
    __shared__ AT lds[kNT / kWave + 1];
    const int64_t n = dc.get();
    const int64_t count = (n + kTile - 1) / kTile;
    AT run = 0;
    for (int64_t b = 0; b < count; b += kNT) {
        const int64_t e = b + threadIdx.x;
        const AT v = e < count ? sums[e] : AT(0);
        AT tot;
        const AT ex = block_excl_scan<kNT>(v, lds, &tot);
        if (e < count) sums[e] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) {
        if (total) *total = run;
        if (at_end) out[n] = run;
    }
}

template <typename IT, typename AT>
__global__ void __launch_bounds__(kNT)
tile_scan_dev_kernel(const IT* __restrict__ in, DevCount dc, const AT* __restrict__ sums,
                     AT* __restrict__ out) {
    __shared__ AT lds[kNT / kWave + 1];
    const int64_t n = dc.get();
    const int64_t tiles = (n + kTile - 1) / kTile;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t base = t * kTile;
        AT run = sums[t];
        for (int i = 0; i < kItems; i++) {
            const int64_t e = base + (int64_t)i * kNT + threadIdx.x;
            const AT v = e < n ? (AT)in[e] : AT(0);
            AT tot;
            const AT ex = block_excl_scan<kNT>(v, lds, &tot);
            if (e < n) out[e] = run + ex;
            run += tot;
        }
    }
}

template <typename IT, typename AT>
pg_status exclusive_scan_dev(const IT* in, AT* out, const uint32_t* cnt, uint32_t mul, uint32_t add,
                             int64_t n_max, AT* total, bool at_end, AT* sums, hipStream_t s) {
    const int64_t tiles = n_max > 0 ? (n_max + kTile - 1) / kTile : 1;
    const unsigned grid = (unsigned)(tiles < 1024 ? tiles : 1024);
    const DevCount dc{cnt, mul, add};
    hipLaunchKernelGGL((tile_sum_dev_kernel<IT, AT>), dim3(grid), dim3(kNT), 0, s, in, dc, sums);
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL((scan_sums_dev_kernel<AT>), dim3(1), dim3(kNT), 0, s, sums, dc, total, out,
                       at_end ? 1 : 0);
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL((tile_scan_dev_kernel<IT, AT>), dim3(grid), dim3(kNT), 0, s, in, dc, sums, out);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

__global__ void fill_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

int64_t scan_partials(int64_t n) { return n > 0 ? (n + kTile - 1) / kTile : 1; }

pg_status exclusive_scan_u32_ws(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                                uint32_t* sums, hipStream_t s) {
    return exclusive_scan_ws<uint32_t, uint32_t>(in, out, n, total, sums, s);
}

pg_status fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return PG_OK;
    hipLaunchKernelGGL(fill_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s, p, n, v);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

pg_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                             hipStream_t s) {
    return exclusive_scan<uint32_t, uint32_t>(in, out, n, total, s);
}

pg_status exclusive_scan_i32_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* total,
                                 hipStream_t s) {
    return exclusive_scan<int32_t, int64_t>(in, out, n, total, s);
}

pg_status exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total,
                             hipStream_t s) {
    return exclusive_scan<uint64_t, uint64_t>(in, out, n, total, s);
}

pg_status exclusive_scan_u64_ws(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total,
                                uint64_t* sums, hipStream_t s) {
    return exclusive_scan_ws<uint64_t, uint64_t>(in, out, n, total, sums, s);
}

pg_status exclusive_scan_u32_dev(const uint32_t* in, uint32_t* out, const uint32_t* cnt, uint32_t mul,
                                 uint32_t add, int64_t n_max, uint32_t* total, bool at_end,
                                 uint32_t* sums, hipStream_t s) {
    return exclusive_scan_dev<uint32_t, uint32_t>(in, out, cnt, mul, add, n_max, total, at_end, sums, s);
}

pg_status exclusive_scan_u64_dev(const uint64_t* in, uint64_t* out, const uint32_t* cnt, uint32_t mul,
                                 uint32_t add, int64_t n_max, uint64_t* total, bool at_end,
                                 uint64_t* sums, hipStream_t s) {
    return exclusive_scan_dev<uint64_t, uint64_t>(in, out, cnt, mul, add, n_max, total, at_end, sums, s);
}

}  // namespace pg
