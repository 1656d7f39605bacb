// Exclusive prefix sums (three passes: block totals, scan of the totals,
// block-local scan plus offset) and fill kernels. Deterministic: integer
// sums in a fixed order.
#include "launch.h"

namespace petar {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ int64_t block_excl_scan(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kScanThreads / kWave];
    int64_t incl = wave_incl_scan(v);
    int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int64_t off = 0, tot = 0;
    for (int k = 0; k < kScanThreads / kWave; k++) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

template <typename In>
__global__ __launch_bounds__(kScanThreads) void k_block_totals(const In *in, int64_t n,
                                                               int64_t *bsum) {
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t v = 0;
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) v += (int64_t)in[i];
    }
    int64_t tot;
    block_excl_scan(v, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of nb block totals by one block, in chunks of kScanThreads.
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(int64_t *bsum, int64_t nb) {
    int64_t carry = 0;
    for (int64_t c = 0; c < nb; c += kScanThreads) {
        int64_t i = c + threadIdx.x;
        int64_t v = i < nb ? bsum[i] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan(v, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

template <typename In, typename Out>
__global__ __launch_bounds__(kScanThreads) void k_block_scan(const In *in, Out *out, int64_t n,
                                                             const int64_t *bsum, int64_t nb) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t vals[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + k;
        vals[k] = i < n ? (int64_t)in[i] : 0;
        s += vals[k];
    }
    int64_t tot;
    int64_t off = block_excl_scan(s, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + k;
        if (i < n) out[i] = (Out)off;
        off += vals[k];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = (Out)bsum[nb];
}

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename In, typename Out>
void scan_impl(const In *in, Out *out, int64_t n, int64_t *ws, hipStream_t s) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_block_totals<In>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, ws);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, s, ws, nb);
    hipLaunchKernelGGL((k_block_scan<In, Out>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in,
                       out, n, (const int64_t *)ws, nb);
}

template <typename T>
void fill_impl(T *p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

}  // namespace

int64_t scan_ws_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 2; }

void scan_u32_to_i64(const uint32_t *in, int64_t *out, int64_t n, int64_t *ws, hipStream_t s) {
    scan_impl(in, out, n, ws, s);
}
void scan_u32_to_u32(const uint32_t *in, uint32_t *out, int64_t n, int64_t *ws, hipStream_t s) {
    scan_impl(in, out, n, ws, s);
}
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) { fill_impl(p, v, n, s); }
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) { fill_impl(p, v, n, s); }

}  // namespace petar
