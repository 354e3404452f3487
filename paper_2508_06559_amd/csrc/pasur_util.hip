// pasur_util.hip -- error reporting and the device-wide exclusive scan used
// to lay out tree levels (counts -> CSR offsets).
#include "pasur_internal.hpp"

#include <cstring>

namespace pasur {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;

// Block-wide exclusive scan of one int64 per thread (Hillis-Steele in LDS).
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *total) {
  __shared__ int64_t buf[2][kBlock];
  int t = threadIdx.x;
  int cur = 0;
  buf[cur][t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    int64_t x = buf[cur][t];
    if (t >= off) x += buf[cur][t - off];
    buf[cur ^ 1][t] = x;
    cur ^= 1;
    __syncthreads();
  }
  int64_t incl = buf[cur][t];
  *total = buf[cur][kBlock - 1];
  __syncthreads();
  return incl - v;
}

template <class In>
__global__ void __launch_bounds__(kBlock) k_tile_sums(const In *in, int64_t n, int64_t *sums) {
  int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int64_t s = 0;
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    if (i < n) s += (int64_t)in[i];
  }
  int64_t total;
  (void)block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// out[i] = tile_off[tile] + exclusive prefix inside the tile; the last tile
// also writes out[n] (the grand total).
template <class In>
__global__ void __launch_bounds__(kBlock) k_tile_scan(const In *in, int64_t n,
                                                     const int64_t *tile_off, int64_t *out) {
  int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int64_t v[kItems];
  int64_t s = 0;
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? (int64_t)in[i] : 0;
    s += v[k];
  }
  int64_t total;
  int64_t pre = block_exclusive_scan(s, &total);
  int64_t off = tile_off ? tile_off[blockIdx.x] : 0;
  int64_t run = off + pre;
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + total;
}

template <class In>
int scan_i64(const In *d_in, int64_t n, int64_t *d_out, hipStream_t stream) {
  int64_t nt = (n + kTile - 1) / kTile;
  if (nt <= 1) {
    k_tile_scan<In><<<1, kBlock, 0, stream>>>(d_in, n, nullptr, d_out);
    PASUR_TRY_HIP(hipGetLastError());
    return PASUR_OK;
  }
  int64_t *sums = nullptr, *offs = nullptr;
  PASUR_TRY(dev_alloc(&sums, nt));
  int st = dev_alloc(&offs, nt + 1);
  if (st) { dev_free(sums); return st; }
  k_tile_sums<In><<<(unsigned)nt, kBlock, 0, stream>>>(d_in, n, sums);
  st = scan_i64<int64_t>(sums, nt, offs, stream);
  if (!st) {
    k_tile_scan<In><<<(unsigned)nt, kBlock, 0, stream>>>(d_in, n, offs, d_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("scan launch: %s", hipGetErrorString(e)); st = PASUR_E_HIP; }
  }
  // frees are ordered after the stream's work by the synchronisation below
  hipError_t e = hipStreamSynchronize(stream);
  dev_free(sums);
  dev_free(offs);
  if (!st && e != hipSuccess) { set_error("scan: %s", hipGetErrorString(e)); st = PASUR_E_HIP; }
  return st;
}

__global__ void k_narrow(const int64_t *in, int64_t n, int32_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) out[i] = (int32_t)in[i];
}

}  // namespace

int scan_counts(const int32_t *d_counts, int64_t n, int32_t *d_out,
                int64_t *total, hipStream_t stream) {
  int64_t *tmp = nullptr;
  PASUR_TRY(dev_alloc(&tmp, n + 1));
  int st = scan_i64<int32_t>(d_counts, n, tmp, stream);
  if (!st) {
    hipError_t e = hipMemcpyAsync(total, tmp + n, sizeof(int64_t),
                                  hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) { set_error("scan total: %s", hipGetErrorString(e)); st = PASUR_E_HIP; }
  }
  if (!st && *total > INT32_MAX) {
    set_error("tree level of %lld nodes exceeds INT32_MAX", (long long)*total);
    st = PASUR_E_OVERFLOW;
  }
  if (!st) {
    k_narrow<<<(unsigned)((n + 1 + 255) / 256), 256, 0, stream>>>(tmp, n, d_out);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) { set_error("scan narrow: %s", hipGetErrorString(e)); st = PASUR_E_HIP; }
  }
  dev_free(tmp);
  return st;
}

}  // namespace pasur

extern "C" const char *pasur_last_error(void) { return pasur::g_err; }
extern "C" int pasur_version(void) { return 1; }
