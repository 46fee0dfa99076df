// wcc_prims.hip -- device-wide primitives used by the WCC front end and drivers:
// exclusive prefix sums (int32 / int64) and a stable LSD radix sort of (key, value)
// pairs.  Three-phase tile scan; radix passes of up to 8 bits with stable in-tile
// ranking by wavefront ballots.
#include "wcc_common.h"

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_tile_reduce(const T *in, int64_t n, T *partial) {
  __shared__ T red[SCAN_BLOCK / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    int64_t j = base + (int64_t)i * SCAN_BLOCK + threadIdx.x;
    if (j < n) s += in[j];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if (__lane_id() == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    T t = 0;
    for (int w = 0; w < SCAN_BLOCK / 64; w++) t += red[w];
    partial[blockIdx.x] = t;
  }
}

// one block: exclusive scan of the tile partials, in place; total to *total
template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_partials(T *partial, int64_t np, T *total) {
  __shared__ T red[SCAN_BLOCK / 64 + 1];
  __shared__ T carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < np; base += SCAN_BLOCK) {
    int64_t j = base + threadIdx.x;
    T v = j < np ? partial[j] : 0;
    T inc = v;
    unsigned l = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      T t = __shfl_up(inc, d, 64);
      if (l >= (unsigned)d) inc += t;
    }
    if (l == 63) red[threadIdx.x >> 6] = inc;
    __syncthreads();
    T wbase = 0, all = 0;
    for (int w = 0; w < SCAN_BLOCK / 64; w++) {
      if (w < (int)(threadIdx.x >> 6)) wbase += red[w];
      all += red[w];
    }
    T c = carry;
    if (j < np) partial[j] = c + wbase + inc - v;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + all;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_tile_scan(const T *in, T *out, int64_t n,
                                                          const T *partial) {
  __shared__ T buf[SCAN_TILE];
  __shared__ T red[SCAN_BLOCK / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    int64_t j = base + (int64_t)i * SCAN_BLOCK + threadIdx.x;
    buf[i * SCAN_BLOCK + threadIdx.x] = j < n ? in[j] : 0;
  }
  __syncthreads();
  T loc[SCAN_ITEMS];
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    loc[i] = s;
    s += buf[threadIdx.x * SCAN_ITEMS + i];
  }
  T inc = s;
  unsigned l = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T t = __shfl_up(inc, d, 64);
    if (l >= (unsigned)d) inc += t;
  }
  if (l == 63) red[threadIdx.x >> 6] = inc;
  __syncthreads();
  T wbase = 0;
  for (int w = 0; w < (int)(threadIdx.x >> 6); w++) wbase += red[w];
  T off = partial[blockIdx.x] + wbase + inc - s;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) buf[threadIdx.x * SCAN_ITEMS + i] = off + loc[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; i++) {
    int64_t j = base + (int64_t)i * SCAN_BLOCK + threadIdx.x;
    if (j < n) out[j] = buf[i * SCAN_BLOCK + threadIdx.x];
  }
}

template <typename T>
int excl_scan(const T *in, T *out, int64_t n, T *total_dev, void *tmp, size_t tmp_bytes,
              hipStream_t s) {
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (tiles < 1) tiles = 1;
  if ((size_t)tiles * sizeof(T) > tmp_bytes) return WCC_EINVAL;
  T *partial = (T *)tmp;
  if (n > 0) {
    hipLaunchKernelGGL(k_tile_reduce<T>, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, in, n,
                       partial);
  } else {
    int rc = prim_fill32(partial, 0u, (int64_t)(sizeof(T) / 4), s);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(SCAN_BLOCK), 0, s, partial, tiles,
                     total_dev);
  if (n > 0)
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, in, out,
                       n, (const T *)partial);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_BLOCK = 256;
constexpr int RS_ITERS = 8;
constexpr int RS_TILE = RS_BLOCK * RS_ITERS;

// A pass is inactive when a device-side maximum key is given and has no bits at `shift`;
// an inactive pass copies its input to its output so the buffer parity is unchanged.
DEV bool pass_active(const int32_t *maxkey_m1, int shift) {
  return !maxkey_m1 || ((uint32_t)(*maxkey_m1 + 1) >> shift) != 0;
}

__global__ void __launch_bounds__(RS_BLOCK) k_radix_hist(const uint32_t *keys, int64_t n,
                                                         int shift, uint32_t mask,
                                                         int32_t *hist, int ntiles,
                                                         const int32_t *maxkey_m1) {
  if (!pass_active(maxkey_m1, shift)) return;
  __shared__ int cnt[256];
  for (int d = threadIdx.x; d < 256; d += RS_BLOCK) cnt[d] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int i = 0; i < RS_ITERS; i++) {
    int64_t j = base + (int64_t)i * RS_BLOCK + threadIdx.x;
    if (j < n) atomicAdd(&cnt[(keys[j] >> shift) & mask], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d <= (int)mask; d += RS_BLOCK) hist[(int64_t)d * ntiles + blockIdx.x] = cnt[d];
}

__global__ void __launch_bounds__(RS_BLOCK) k_radix_scatter(const uint32_t *kin, const uint32_t *vin,
                                                            uint32_t *kout, uint32_t *vout,
                                                            int64_t n, int shift, int nbits,
                                                            const int32_t *offs, int ntiles,
                                                            const int32_t *maxkey_m1) {
  constexpr int NW = RS_BLOCK / 64;
  if (!pass_active(maxkey_m1, shift)) {
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int i = threadIdx.x; i < RS_TILE; i += RS_BLOCK)
      if (base + i < n) {
        kout[base + i] = kin[base + i];
        vout[base + i] = vin[base + i];
      }
    return;
  }
  __shared__ int run[256];
  __shared__ int wcnt[NW][256];
  uint32_t mask = (1u << nbits) - 1;
  for (int d = threadIdx.x; d < 256; d += RS_BLOCK)
    run[d] = d <= (int)mask ? offs[(int64_t)d * ntiles + blockIdx.x] : 0;
  int w = threadIdx.x >> 6;
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int it = 0; it < RS_ITERS; it++) {
    for (int j = threadIdx.x; j < NW * 256; j += RS_BLOCK) (&wcnt[0][0])[j] = 0;
    __syncthreads();
    int64_t idx = base + (int64_t)it * RS_BLOCK + threadIdx.x;
    bool valid = idx < n;
    uint32_t k = valid ? kin[idx] : 0u, v = valid ? vin[idx] : 0u;
    uint32_t digit = (k >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; b++) {
      bool bit = (digit >> b) & 1u;
      uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    int rank = __popcll(peers & lanemask_lt());
    if (valid && rank == 0) wcnt[w][digit] = __popcll(peers);
    __syncthreads();
    for (int d = threadIdx.x; d <= (int)mask; d += RS_BLOCK) {
      int s = run[d];
      for (int q = 0; q < NW; q++) {
        int t = wcnt[q][d];
        wcnt[q][d] = s;
        s += t;
      }
      run[d] = s;
    }
    __syncthreads();
    if (valid) {
      int pos = wcnt[w][digit] + rank;
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
  }
}

__global__ void k_fill32(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

// Fills nwords 32-bit words with v (a kernel, so that it can be captured in a graph).
int prim_fill32(void *p, uint32_t v, int64_t nwords, hipStream_t s) {
  if (nwords <= 0) return WCC_OK;
  if ((uintptr_t)p < 65536) return WCC_EINVAL;  // an unallocated buffer (plus an offset)
  int64_t blocks = (nwords + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p, v, nwords);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

size_t prim_scan_tmp_bytes(int64_t n) {
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (tiles < 1) tiles = 1;
  return (size_t)(tiles + 1) * sizeof(int64_t);
}

int prim_excl_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev, void *tmp,
                       size_t tmp_bytes, hipStream_t s) {
  return excl_scan<int32_t>(in, out, n, total_dev, tmp, tmp_bytes, s);
}
int prim_excl_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *tmp,
                       size_t tmp_bytes, hipStream_t s) {
  return excl_scan<int64_t>(in, out, n, total_dev, tmp, tmp_bytes, s);
}

size_t prim_radix_tmp_bytes(int64_t n) {
  int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
  if (tiles < 1) tiles = 1;
  size_t hist = (size_t)tiles * 256 * sizeof(int32_t);
  return 2 * hist + prim_scan_tmp_bytes(tiles * 256) + 256;
}

// Stable sort of (keys, vals) by the low `bits` bits of the keys.  The result ends in
// (keys, vals) or in the alternates (*result_in_alt = 1).
int prim_radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                          int64_t n, int bits, void *tmp, size_t tmp_bytes, hipStream_t s,
                          int *result_in_alt, const int32_t *maxkey_m1) {
  *result_in_alt = 0;
  if (n <= 1 || bits <= 0) return WCC_OK;
  if (tmp_bytes < prim_radix_tmp_bytes(n)) return WCC_EINVAL;
  int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
  int32_t *hist = (int32_t *)tmp;
  int32_t *offs = hist + (size_t)ntiles * 256;
  void *stmp = (void *)(offs + (size_t)ntiles * 256);
  size_t stmp_bytes = tmp_bytes - 2 * (size_t)ntiles * 256 * sizeof(int32_t);
  uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
  for (int shift = 0; shift < bits; shift += 8) {
    int nb = bits - shift < 8 ? bits - shift : 8;
    uint32_t mask = (1u << nb) - 1;
    int64_t hn = (int64_t)(mask + 1) * ntiles;
    hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(RS_BLOCK), 0, s, (const uint32_t *)ki, n,
                       shift, mask, hist, ntiles, maxkey_m1);
    int rc = prim_excl_scan_i32(hist, offs, hn, nullptr, stmp, stmp_bytes, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(RS_BLOCK), 0, s, (const uint32_t *)ki,
                       (const uint32_t *)vi, ko, vo, n, shift, nb, (const int32_t *)offs, ntiles, maxkey_m1);
    HIP_TRY(hipGetLastError());
    uint32_t *t = ki;
    ki = ko;
    ko = t;
    t = vi;
    vi = vo;
    vo = t;
    *result_in_alt ^= 1;
  }
  return WCC_OK;
}
