// pasur_sort.hip -- stable LSD radix sort of (key, int32 value) pairs, used by
// the unfolding to group leaves by their next-round root (the canonical
// (compressed pool, score) key of section "Between-Hand Updates") and root
// scores by their score key.
//
// One pass per 8-bit digit that actually varies over the keys (an AND/OR
// reduction finds them first).  A pass is three launches:
//   k_rs_hist     per 4096-key tile, a 256-bucket histogram in LDS, stored
//                 digit-major: hist[d * n_tiles + tile];
//   scan_counts   exclusive scan of that array: the first output slot of
//                 (digit d, tile) in the sorted order;
//   k_rs_scatter  per tile, the stable rank of every key within its digit
//                 (wavefront ballots over the digit's bits give the rank
//                 among equal digits of one wave; per-wave counts in LDS
//                 order the waves and the tile's 16 rounds), then the tile is
//                 reordered in LDS by digit so that each bucket's run leaves
//                 as consecutive addresses.
#include "pasur_internal.hpp"

namespace pasur {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;
constexpr int kBuckets = 256;

template <class K>
__global__ void __launch_bounds__(kBlock) k_rs_andor(const K *__restrict__ keys, int64_t n,
                                                     unsigned long long *__restrict__ acc) {
  K a = ~K(0), o = K(0);
  const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + (int64_t)r * kBlock;
    if (i < n) {
      const K k = keys[i];
      a &= k;
      o |= k;
    }
  }
  __shared__ unsigned long long sa[kBlock], so[kBlock];
  sa[threadIdx.x] = (unsigned long long)a;
  so[threadIdx.x] = (unsigned long long)o;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sa[threadIdx.x] &= sa[threadIdx.x + s];
      so[threadIdx.x] |= so[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAnd(&acc[0], sa[0]);
    atomicOr(&acc[1], so[0]);
  }
}

__global__ void k_rs_andor_init(unsigned long long *acc) {
  if (threadIdx.x == 0) {
    acc[0] = ~0ull;
    acc[1] = 0ull;
  }
}

template <class K>
__global__ void __launch_bounds__(kBlock) k_rs_hist(const K *__restrict__ keys, int64_t n,
                                                    int shift, int64_t n_tiles,
                                                    int32_t *__restrict__ hist) {
  __shared__ int32_t h[kBuckets];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + (int64_t)r * kBlock;
    if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & 0xFF)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

template <class K>
__global__ void __launch_bounds__(kBlock) k_rs_scatter(const K *__restrict__ keys,
                                                       const int32_t *__restrict__ vals, int64_t n,
                                                       int shift, int64_t n_tiles,
                                                       const int32_t *__restrict__ off,
                                                       K *__restrict__ okeys,
                                                       int32_t *__restrict__ ovals) {
  __shared__ int32_t cnt[kBuckets];         // keys of each digit in earlier rounds
  __shared__ int32_t wc[kWaves][kBuckets];  // this round's count per wave and digit
  __shared__ int32_t loc[2][kBuckets];      // tile-local exclusive offsets (scan buffers)
  __shared__ int32_t gof[kBuckets];         // this tile's first output slot per digit
  __shared__ K sk[kTile];
  __shared__ int32_t sv[kTile];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int count = (int)(n - base < kTile ? n - base : kTile);
  cnt[t] = 0;
  gof[t] = off[(int64_t)t * n_tiles + blockIdx.x];
  K k[kItems];
  int32_t v[kItems];
  int rank[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int i = r * kBlock + t;
    k[r] = i < count ? keys[base + i] : K(0);
    v[r] = i < count ? vals[base + i] : 0;
  }
  const unsigned long long below_mask = (1ull << lane) - 1;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
#pragma unroll
    for (int q = 0; q < kWaves; ++q) wc[q][t] = 0;
    __syncthreads();
    const bool ok = r * kBlock + t < count;
    const int d = (int)((k[r] >> shift) & 0xFF);
    unsigned long long m = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long bb = __ballot((d >> b) & 1);
      m &= ((d >> b) & 1) ? bb : ~bb;
    }
    const int below = __popcll(m & below_mask);
    if (ok && below == 0) wc[w][d] = __popcll(m);
    __syncthreads();
    int pre = cnt[d];
    for (int q = 0; q < w; ++q) pre += wc[q][d];
    rank[r] = pre + below;
    __syncthreads();
    cnt[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
  }
  // tile-local exclusive offsets of the digits (Hillis-Steele over 256)
  int cur = 0;
  loc[0][t] = cnt[t];
  __syncthreads();
  for (int s = 1; s < kBuckets; s <<= 1) {
    int x = loc[cur][t];
    if (t >= s) x += loc[cur][t - s];
    loc[cur ^ 1][t] = x;
    cur ^= 1;
    __syncthreads();
  }
  const int excl = loc[cur][t] - cnt[t];
  __syncthreads();
  loc[cur ^ 1][t] = excl;
  __syncthreads();
  const int *lo = loc[cur ^ 1];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    if (r * kBlock + t < count) {
      const int d = (int)((k[r] >> shift) & 0xFF);
      const int p = lo[d] + rank[r];
      sk[p] = k[r];
      sv[p] = v[r];
    }
  }
  __syncthreads();
  for (int j = t; j < count; j += kBlock) {
    const K kk = sk[j];
    const int d = (int)((kk >> shift) & 0xFF);
    const int64_t g = (int64_t)gof[d] + (j - lo[d]);
    okeys[g] = kk;
    ovals[g] = sv[j];
  }
}

unsigned grid_tiles(int64_t n) { return (unsigned)((n + kTile - 1) / kTile); }

}  // namespace

template <class K>
int radix_sort_pairs(K *keys, K *keys_out, int32_t *vals, int32_t *vals_out, int64_t n,
                     int end_bit, hipStream_t s) {
  if (n <= 0) return PASUR_OK;
  const int64_t n_tiles = (n + kTile - 1) / kTile;
  unsigned long long *acc = nullptr;
  PASUR_TRY(dev_alloc(&acc, 2));
  k_rs_andor_init<<<1, 64, 0, s>>>(acc);
  k_rs_andor<K><<<grid_tiles(n), kBlock, 0, s>>>(keys, n, acc);
  unsigned long long h_acc[2] = {0, 0};
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h_acc, acc, sizeof(h_acc), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(acc);
  if (e != hipSuccess) {
    set_error("radix sort: %s", hipGetErrorString(e));
    return PASUR_E_HIP;
  }
  const unsigned long long varying = h_acc[0] ^ h_acc[1];
  int shifts[8], n_pass = 0;
  for (int sh = 0; sh < end_bit && sh < 8 * (int)sizeof(K); sh += 8)
    if ((varying >> sh) & 0xFF) shifts[n_pass++] = sh;
  K *ks[2] = {keys, keys_out};
  int32_t *vs[2] = {vals, vals_out};
  int src = 0;
  int st = PASUR_OK;
  if (n_pass > 0) {
    int32_t *hist = nullptr, *off = nullptr;
    st = dev_alloc(&hist, n_tiles * kBuckets);
    if (!st) st = dev_alloc(&off, n_tiles * kBuckets + 1);
    for (int p = 0; p < n_pass && !st; ++p) {
      k_rs_hist<K><<<grid_tiles(n), kBlock, 0, s>>>(ks[src], n, shifts[p], n_tiles, hist);
      e = hipGetLastError();
      if (e != hipSuccess) {
        set_error("radix sort: %s", hipGetErrorString(e));
        st = PASUR_E_HIP;
        break;
      }
      int64_t total = 0;
      st = scan_counts(hist, n_tiles * kBuckets, off, &total, s);
      if (st) break;
      k_rs_scatter<K><<<grid_tiles(n), kBlock, 0, s>>>(ks[src], vs[src], n, shifts[p], n_tiles,
                                                       off, ks[src ^ 1], vs[src ^ 1]);
      e = hipGetLastError();
      if (e != hipSuccess) {
        set_error("radix sort: %s", hipGetErrorString(e));
        st = PASUR_E_HIP;
      }
      src ^= 1;
    }
    e = hipStreamSynchronize(s);
    dev_free(hist);
    dev_free(off);
    if (!st && e != hipSuccess) {
      set_error("radix sort: %s", hipGetErrorString(e));
      st = PASUR_E_HIP;
    }
  }
  if (!st && src == 0) {  // the sorted pairs are in the input buffers
    e = hipMemcpyAsync(keys_out, keys, n * sizeof(K), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(vals_out, vals, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      set_error("radix sort: %s", hipGetErrorString(e));
      st = PASUR_E_HIP;
    }
  }
  return st;
}

template int radix_sort_pairs<uint32_t>(uint32_t *, uint32_t *, int32_t *, int32_t *, int64_t,
                                        int, hipStream_t);
template int radix_sort_pairs<uint64_t>(uint64_t *, uint64_t *, int32_t *, int32_t *, int64_t,
                                        int, hipStream_t);

}  // namespace pasur
