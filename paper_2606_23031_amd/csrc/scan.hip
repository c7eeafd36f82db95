// Device-wide exclusive scan (reduce-then-scan) for uint32 counts.
#include "dv_internal.h"

namespace dv {

constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = TPB * SCAN_ITEMS;   // 4096 counts per block

// Inclusive wave64 scan with shuffles.
template <class T>
__device__ inline T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

// Exclusive block scan of one value per thread (256 threads).
template <class T>
__device__ inline T block_excl_scan(T v, T* lds4, T* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T inc = wave_incl_scan(v);
  if (lane == 63) lds4[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < TPB / 64; ++i) {
    T x = lds4[i];
    if (i < w) off += x;
    tot += x;
  }
  __syncthreads();
  if (total) *total = tot;
  return off + inc - v;
}

__global__ void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                              uint64_t* __restrict__ part) {
  __shared__ uint64_t lds[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + (int64_t)i * TPB + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  // block reduction
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) lds[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

__global__ void k_scan_partials(uint64_t* __restrict__ part, int64_t nb,
                                uint64_t* __restrict__ total) {
  __shared__ uint64_t lds[4];
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += TPB) {
    int64_t i = base + threadIdx.x;
    uint64_t v = i < nb ? part[i] : 0;
    uint64_t tot;
    uint64_t ex = block_excl_scan<uint64_t>(v, lds, &tot);
    if (i < nb) part[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void k_scan_apply(const uint32_t* __restrict__ in, int64_t n,
                             const uint64_t* __restrict__ part,
                             uint32_t* __restrict__ out) {
  __shared__ uint64_t lds[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE +
                       (int64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    v[i] = idx < n ? in[idx] : 0u;
    s += v[i];
  }
  uint64_t off = block_excl_scan<uint64_t>(s, lds, nullptr) + part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = (uint32_t)off;
    off += v[i];
  }
}

dv_status exclusive_scan_u32(dv_ctx* ctx, const uint32_t* in, uint32_t* out,
                             uint64_t* total_dev, int64_t n, hipStream_t s) {
  if (n <= 0) {
    if (total_dev) {
      hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(TPB), 0, s,
                         (uint64_t*)nullptr, (int64_t)0, total_dev);
      DV_TRY_HIP(hipGetLastError());
    }
    return DV_OK;
  }
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  DBuf part;
  DV_TRY(alloc_n<uint64_t>(ctx, part, nb, s));
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(TPB), 0, s, in,
                     n, part.as<uint64_t>());
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(TPB), 0, s,
                     part.as<uint64_t>(), nb, total_dev);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(TPB), 0, s, in, n,
                     part.as<uint64_t>(), out);
  DV_TRY_HIP(hipGetLastError());
  return DV_OK;
}

}  // namespace dv
