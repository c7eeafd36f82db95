// Stable LSD radix sort of (key, value) pairs, 8- or 9-bit digits (the
// width that needs fewer passes over the key bits; 8 on a tie).
//
// Each pass: per-block digit histograms (LDS atomics), a device scan of the
// digit-major count matrix, and a stable scatter.  In the scatter every
// wave64 ranks its 64 keys per round with ballots (one ballot per digit
// bit gives the set of lanes holding the same digit), keeps running
// per-wave digit counters in LDS, then offsets waves within the block.
// Element order inside a block is (wave, round, lane), so equal digits keep
// their input order and the sort is stable.
#include "dv_internal.h"

namespace dv {

constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = TPB * RS_ITEMS;     // 4096 keys per block
constexpr int RS_WAVE_SPAN = 64 * RS_ITEMS;  // 1024 keys per wave

template <class K, int DB>
__global__ void __launch_bounds__(TPB)
k_rs_hist(const K* __restrict__ keys, int64_t n, int sh,
          uint32_t* __restrict__ counts, int64_t nb) {
  constexpr int BINS = 1 << DB;
  constexpr uint32_t MASK = BINS - 1;
  __shared__ uint32_t hist[BINS];
  for (int d = threadIdx.x; d < BINS; d += TPB) hist[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    int64_t idx = base + (int64_t)i * TPB + threadIdx.x;
    if (idx < n) {
      uint32_t d = (uint32_t)(keys[idx] >> sh) & MASK;
      atomicAdd(&hist[d], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < BINS; d += TPB)
    counts[(int64_t)d * nb + blockIdx.x] = hist[d];
}

template <class K, int DB>
__global__ void __launch_bounds__(TPB)
k_rs_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
             K* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n,
             int sh, const uint32_t* __restrict__ offs, int64_t nb) {
  constexpr int BINS = 1 << DB;
  constexpr uint32_t MASK = BINS - 1;
  __shared__ uint32_t wcnt[TPB / 64][BINS];
  __shared__ uint32_t wbase[TPB / 64][BINS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < BINS; d += TPB)
#pragma unroll
    for (int i = 0; i < TPB / 64; ++i) wcnt[i][d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * RS_WAVE_SPAN;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  K key[RS_ITEMS];
  uint32_t val[RS_ITEMS], pos[RS_ITEMS], dig[RS_ITEMS];
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    const bool valid = idx < n;
    K k = valid ? kin[idx] : (K)0;
    uint32_t v = valid ? vin[idx] : 0u;
    uint32_t d = (uint32_t)(k >> sh) & MASK;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < DB; ++b) {
      const bool bit = (d >> b) & 1;
      uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t r = (uint32_t)__popcll(peers & lt);
    const uint32_t c0 = wcnt[w][d];
    __builtin_amdgcn_wave_barrier();
    if (valid && r == 0) wcnt[w][d] = c0 + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    key[j] = k;
    val[j] = v;
    dig[j] = valid ? d : 0xFFFFFFFFu;
    pos[j] = c0 + r;
  }
  __syncthreads();
  for (int d = threadIdx.x; d < BINS; d += TPB) {
    uint32_t off = offs[(int64_t)d * nb + blockIdx.x];
#pragma unroll
    for (int i = 0; i < TPB / 64; ++i) {
      wbase[i][d] = off;
      off += wcnt[i][d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    if (dig[j] != 0xFFFFFFFFu) {
      const uint32_t dst = wbase[w][dig[j]] + pos[j];
      kout[dst] = key[j];
      vout[dst] = val[j];
    }
  }
}

template <class K>
static dv_status radix_sort(dv_ctx* ctx, K* keys, uint32_t* vals, K* kalt,
                            uint32_t* valt, int64_t n, int bits,
                            hipStream_t s, bool* in_alt) {
  *in_alt = false;
  if (n <= 1 || bits <= 0) return DV_OK;
  if (n >= (int64_t)0xFFFFFFFFll) {
    set_error("radix sort: %lld elements exceed the 32-bit index range",
              (long long)n);
    return DV_ERR_LIMIT;
  }
  const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
  // 9-bit digits where they save a pass (18 bits: 2 passes, not 3)
  const bool wide = (bits + 8) / 9 < (bits + 7) / 8;
  const int db = wide ? 9 : 8;
  const int64_t bins = (int64_t)1 << db;
  DBuf cnt, off;
  DV_TRY(alloc_n<uint32_t>(ctx, cnt, nb * bins, s));
  DV_TRY(alloc_n<uint32_t>(ctx, off, nb * bins, s));
  K* ka = keys;
  uint32_t* va = vals;
  K* kb = kalt;
  uint32_t* vb = valt;
  auto hist = wide ? k_rs_hist<K, 9> : k_rs_hist<K, 8>;
  auto scatter = wide ? k_rs_scatter<K, 9> : k_rs_scatter<K, 8>;
  for (int sh = 0; sh < bits; sh += db) {
    hipLaunchKernelGGL(hist, dim3((unsigned)nb), dim3(TPB), 0, s, ka, n, sh,
                       cnt.as<uint32_t>(), nb);
    DV_TRY(exclusive_scan_u32(ctx, cnt.as<uint32_t>(), off.as<uint32_t>(),
                              nullptr, nb * bins, s));
    hipLaunchKernelGGL(scatter, dim3((unsigned)nb), dim3(TPB), 0, s, ka, va, kb,
                       vb, n, sh, off.as<uint32_t>(), nb);
    DV_TRY_HIP(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
    *in_alt = !*in_alt;
  }
  return DV_OK;
}

dv_status radix_sort_u64(dv_ctx* ctx, uint64_t* keys, uint32_t* vals,
                         uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                         int bits, hipStream_t s, bool* in_alt) {
  return radix_sort<uint64_t>(ctx, keys, vals, keys_alt, vals_alt, n, bits, s,
                              in_alt);
}

dv_status radix_sort_u32(dv_ctx* ctx, uint32_t* keys, uint32_t* vals,
                         uint32_t* keys_alt, uint32_t* vals_alt, int64_t n,
                         int bits, hipStream_t s, bool* in_alt) {
  return radix_sort<uint32_t>(ctx, keys, vals, keys_alt, vals_alt, n, bits, s,
                              in_alt);
}

}  // namespace dv
