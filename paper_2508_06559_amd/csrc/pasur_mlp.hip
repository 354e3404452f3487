// pasur_mlp.hip -- the learned warm start: a 192-256-256-2 MLP over card
// bitmasks, the inherited score and the score of the round so far, trained on the average strategies and
// node values that the DCFR kernels produce, and used to initialise DCFR on
// new deals.  GEMMs run on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16:
// BF16 operands, FP32 accumulation).
#include "pasur_internal.hpp"

#include <algorithm>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <type_traits>

using namespace pasur;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(uint16_t)))) uint16_t u16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

namespace {

constexpr int kIn = 192, kHid = 256, kOut = 2;
constexpr int kMaxDevices = 64;
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
constexpr int BK = 32, LDK = BK + 8;  // 80-byte LDS rows keep 16-byte alignment

struct GemmArgs {
  int M, N, K;
  const __bf16 *A;
  int64_t sar, sac;  // op(A)(m, k) = A[m * sar + k * sac]
  const __bf16 *B;
  int64_t sbr, sbc;  // op(B)(k, n) = B[k * sbr + n * sbc]
  float *Cf;         // FP32 output (row stride ldc), split-K partial z at Cf + z * split_stride
  __bf16 *Cb;        // BF16 output (row stride ldc), unused with split-K
  int64_t ldc, split_stride;
  const float *bias;  // per output column, may be null
  int relu;
  int kchunk;  // K range of one split (blockIdx.z)
  // ReLU-backward epilogue (split-free products only): C(m, n) is kept where
  // mask[m * ldc + n] > 0 and zeroed elsewhere, and each row tile's column
  // sums of the kept FP32 values go to colpart[blockIdx.y * N + n]
  const __bf16 *mask;
  float *colpart;
};

// One operand tile (ROWS x BK, rows = output rows of A or output columns of
// B) from global memory into LDS T[ROWS][LDK], for op(X)(row, k) =
// X[row * s_row + k * s_k], in two steps so that the global loads of the next
// K step are in flight during the MFMAs of this one: fetch() reads a full
// tile into registers, commit() writes it to LDS.  A full tile whose
// contiguous global direction is K goes with 16-byte loads straight into LDS
// rows.  One whose contiguous direction is the rows takes, per thread, the
// 16-byte runs of eight rows at two consecutive k and writes each row's pair
// (k, k+1) as one 32-bit LDS word: lanes of one k pair and row blocks eight
// rows apart would otherwise all meet in two LDS banks.  Edge tiles and
// unaligned operands are read element by element in commit() (zeros outside
// the matrix and the K range).
template <int ROWS>
struct TileLoader {
  static constexpr int N = ROWS / 64;             // 16-byte loads per thread, K contiguous
  static constexpr int NP = (ROWS / 8) * (BK / 2);  // (row block, k pair) tasks, rows contiguous
  static constexpr int NPT = (NP + 255) / 256;     // such tasks per thread
  static constexpr int NV = N > 2 * NPT ? N : 2 * NPT;
  bf16x8 v[NV];
  int mode;  // 0: K contiguous, 1: rows contiguous, 2: element by element

  __device__ __forceinline__ void fetch(const __bf16 *X, int64_t s_row, int64_t s_k, int row0,
                                        int nrows, int k0, int kend, bool aligned, int tid) {
    const bool full = row0 + ROWS <= nrows && k0 + BK <= kend && aligned;
    mode = (full && s_k == 1 && (s_row & 7) == 0) ? 0 : (full && s_row == 1 && (s_k & 7) == 0) ? 1 : 2;
    if (mode == 0) {
#pragma unroll
      for (int it = 0; it < N; ++it) {
        const int idx = tid + it * 256, r = idx >> 2, c = (idx & 3) * 8;
        v[it] = *reinterpret_cast<const bf16x8 *>(X + (int64_t)(row0 + r) * s_row + (k0 + c));
      }
    } else if (mode == 1) {
#pragma unroll
      for (int it = 0; it < NPT; ++it) {
        const int idx = tid + it * 256;
        if (idx < NP) {
          const int c = 2 * (idx % (BK / 2)), r = (idx / (BK / 2)) * 8;
          const __bf16 *p = X + (int64_t)(k0 + c) * s_k + (row0 + r);
          v[2 * it] = *reinterpret_cast<const bf16x8 *>(p);
          v[2 * it + 1] = *reinterpret_cast<const bf16x8 *>(p + s_k);
        }
      }
    }
  }

  __device__ __forceinline__ void commit(__bf16 (*T)[LDK], const __bf16 *X, int64_t s_row,
                                         int64_t s_k, int row0, int nrows, int k0, int kend,
                                         int tid) const {
    if (mode == 0) {
#pragma unroll
      for (int it = 0; it < N; ++it) {
        const int idx = tid + it * 256, r = idx >> 2, c = (idx & 3) * 8;
        *reinterpret_cast<bf16x8 *>(&T[r][c]) = v[it];
      }
    } else if (mode == 1) {
#pragma unroll
      for (int it = 0; it < NPT; ++it) {
        const int idx = tid + it * 256;
        if (idx < NP) {
          const int c = 2 * (idx % (BK / 2)), r = (idx / (BK / 2)) * 8;
          // bit patterns of whole vectors (a bit cast of one subscripted
          // __bf16 element yields element 0 with this compiler)
          const u16x8 lo = __builtin_bit_cast(u16x8, v[2 * it]);
          const u16x8 hi = __builtin_bit_cast(u16x8, v[2 * it + 1]);
#pragma unroll
          for (int j = 0; j < 8; ++j)
            *reinterpret_cast<uint32_t *>(&T[r + j][c]) = (uint32_t)lo[j] | ((uint32_t)hi[j] << 16);
        }
      }
    } else {
      const __bf16 zero = (__bf16)0.f;
      for (int e = tid; e < ROWS * BK; e += 256) {
        int r, c;
        if (s_k == 1) { r = e / BK; c = e % BK; } else { c = e / ROWS; r = e % ROWS; }
        const int row = row0 + r, k = k0 + c;
        T[r][c] = (row < nrows && k < kend) ? X[row * s_row + k * s_k] : zero;
      }
    }
  }
};

// C = op(A) op(B) (+ bias, ReLU).  Workgroup tile (32 TI) x (32 TJ), K step
// 32; four waves each own a (16 TI) x (16 TJ) quadrant as TI x TJ MFMA
// 16x16x32 tiles.  MFMA operand layout: lane l holds row (l % 16) of the A
// tile and column (l % 16) of the B tile, K elements 8*(l/16) .. 8*(l/16)+7;
// the accumulator holds rows 4*(l/16) .. +3 of column (l % 16).
// MASK selects the ReLU-backward epilogue at compile time (g.mask set), so
// the plain products do not carry its registers.  256-wide tiles (the ReLU
// backward over all columns, so that A is read once) hold 128 accumulators
// per lane and are capped at two waves per SIMD (no spills).
template <int TI, int TJ, bool MASK>
__global__ void __launch_bounds__(256, TJ > 4 ? 2 : 1) k_gemm(GemmArgs g) {
  constexpr int BM = 32 * TI, BN = 32 * TJ;
  __shared__ __align__(16) __bf16 As[BM][LDK];
  __shared__ __align__(16) __bf16 Bs[BN][LDK];
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 16 * TI, wn = (wave & 1) * 16 * TJ;
  f32x4 acc[TI][TJ];
  for (int i = 0; i < TI; ++i)
    for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // 16-byte aligned operands and K-range starts (the fast tile loads need both)
  const bool a_al = ((reinterpret_cast<uintptr_t>(g.A) & 15) == 0) && (kbeg & 7) == 0;
  const bool b_al = ((reinterpret_cast<uintptr_t>(g.B) & 15) == 0) && (kbeg & 7) == 0;
  TileLoader<BM> la;
  TileLoader<BN> lb;
  if (kbeg < kend) {
    la.fetch(g.A, g.sar, g.sac, m0, g.M, kbeg, kend, a_al, tid);
    lb.fetch(g.B, g.sbc, g.sbr, n0, g.N, kbeg, kend, b_al, tid);
  }
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    la.commit(As, g.A, g.sar, g.sac, m0, g.M, k0, kend, tid);
    lb.commit(Bs, g.B, g.sbc, g.sbr, n0, g.N, k0, kend, tid);
    __syncthreads();
    if (k0 + BK < kend) {
      la.fetch(g.A, g.sar, g.sac, m0, g.M, k0 + BK, kend, a_al, tid);
      lb.fetch(g.B, g.sbc, g.sbr, n0, g.N, k0 + BK, kend, b_al, tid);
    }
    bf16x8 a[TI], b[TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
      a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < TJ; ++j)
      b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + j * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  if (!MASK && g.Cb && !g.Cf && gridDim.z == 1 && m0 + BM <= g.M && n0 + BN <= g.N &&
      (g.ldc & 7) == 0 && (reinterpret_cast<uintptr_t>(g.Cb) & 15) == 0) {
    // Full BF16 tile: each wave stages half of its quadrant at a time in LDS
    // (the operand tiles are no longer read) and writes it as 16-byte row
    // pieces, eight lanes per 128-byte run, instead of 2-byte stores.
    constexpr int RH = 8 * TI, CW = 16 * TJ, SS = CW + 8;  // rows per half, columns, stride
    static_assert(MASK || 2 * RH * SS <= BM * LDK, "two waves' halves fit one operand tile");
    __bf16 *S = (wave < 2 ? &As[0][0] : &Bs[0][0]) + (wave & 1) * RH * SS;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int ii = 0; ii < TI / 2; ++ii)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = ii * 16 + 4 * (lane >> 4) + r, col = j * 16 + (lane & 15);
            float v = acc[h * (TI / 2) + ii][j][r];
            if (g.bias) v += g.bias[n0 + wn + col];
            if (g.relu) v = fmaxf(v, 0.f);
            S[row * SS + col] = (__bf16)v;
          }
      __syncthreads();
      for (int c = lane; c < RH * CW / 8; c += 64) {
        const int row = c / (CW / 8), col = (c % (CW / 8)) * 8;
        *reinterpret_cast<bf16x8 *>(g.Cb + (int64_t)(m0 + wm + h * RH + row) * g.ldc + n0 + wn + col) =
            *reinterpret_cast<const bf16x8 *>(S + row * SS + col);
      }
      __syncthreads();
    }
    return;
  }
  if constexpr (MASK) {
    // ReLU backward: mask, BF16 store, and the row tile's column sums (per
    // column: this lane's rows in (i, r) order, then the four lane groups
    // and the two row halves of the tile in a fixed order)
    __shared__ float csum[2][BN];
    float cs[TJ];
#pragma unroll
    for (int j = 0; j < TJ; ++j) cs[j] = 0.f;
    if (m0 + BM <= g.M && n0 + BN <= g.N && (g.ldc & 7) == 0 &&
        ((reinterpret_cast<uintptr_t>(g.Cb) | reinterpret_cast<uintptr_t>(g.mask)) & 15) == 0) {
      // full tile: each wave brings a part (half, or a quarter for 256-wide
      // tiles) of its quadrant's mask into LDS with 16-byte loads, masks its
      // accumulators there in place (each lane its own elements) and writes
      // the part out as 16-byte row pieces
      constexpr int H = TJ > 4 ? 4 : 2;                        // parts per quadrant
      constexpr int RH = 16 * TI / H, CW = 16 * TJ, SS = CW + 8;  // rows per part, columns, stride
      static_assert(2 * RH * SS <= BM * LDK, "two waves' parts fit one operand tile");
      __bf16 *S = (wave < 2 ? &As[0][0] : &Bs[0][0]) + (wave & 1) * RH * SS;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int64_t base = (int64_t)(m0 + wm + h * RH) * g.ldc + n0 + wn;
        for (int c = lane; c < RH * CW / 8; c += 64) {
          const int row = c / (CW / 8), col = (c % (CW / 8)) * 8;
          *reinterpret_cast<bf16x8 *>(S + row * SS + col) =
              *reinterpret_cast<const bf16x8 *>(g.mask + base + (int64_t)row * g.ldc + col);
        }
        __syncthreads();
#pragma unroll
        for (int ii = 0; ii < TI / H; ++ii)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = ii * 16 + 4 * (lane >> 4) + r, col = j * 16 + (lane & 15);
              const float v = (float)S[row * SS + col] > 0.f ? acc[h * (TI / H) + ii][j][r] : 0.f;
              S[row * SS + col] = (__bf16)v;
              cs[j] += v;
            }
        __syncthreads();
        for (int c = lane; c < RH * CW / 8; c += 64) {
          const int row = c / (CW / 8), col = (c % (CW / 8)) * 8;
          *reinterpret_cast<bf16x8 *>(g.Cb + base + (int64_t)row * g.ldc + col) =
              *reinterpret_cast<const bf16x8 *>(S + row * SS + col);
        }
        __syncthreads();
      }
    } else {
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
            const int n = n0 + wn + j * 16 + (lane & 15);
            if (m < g.M && n < g.N) {
              const int64_t o = (int64_t)m * g.ldc + n;
              const float v = (float)g.mask[o] > 0.f ? acc[i][j][r] : 0.f;
              g.Cb[o] = (__bf16)v;
              cs[j] += v;
            }
          }
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      cs[j] += __shfl_xor(cs[j], 16);
      cs[j] += __shfl_xor(cs[j], 32);
    }
    if (lane < 16) {
#pragma unroll
      for (int j = 0; j < TJ; ++j) csum[wave >> 1][wn + j * 16 + lane] = cs[j];
    }
    __syncthreads();
    for (int c = tid; c < BN; c += 256)
      if (n0 + c < g.N) g.colpart[(int64_t)blockIdx.y * g.N + n0 + c] = csum[0][c] + csum[1][c];
    return;
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          float v = acc[i][j][r];
          if (g.bias) v += g.bias[n];
          if (g.relu) v = fmaxf(v, 0.f);
          if (g.Cf) g.Cf[(int64_t)blockIdx.z * g.split_stride + (int64_t)m * g.ldc + n] = v;
          if (g.Cb) g.Cb[(int64_t)m * g.ldc + n] = (__bf16)v;
        }
      }
}

// 128x128 workgroup tiles where both output dimensions reach 128, else 64x64
// (the 2-wide layer and small problems).  Split-K products (weight
// gradients: a few output tiles, long K) take 64x128 tiles when N reaches
// 128: more workgroups in flight than 128x128 and twice the MFMA work per K
// step of 64x64 (per training step of 2^18 rows: 0.80 ms, against 0.89 with
// 64x64 and more with 128x128).
inline bool big_tiles(int M, int N) { return M >= 128 && N >= 128; }
// Row tiles of a split-free product's grid (its blockIdx.y range).
inline int row_tiles(int M, int N) { return (M + (big_tiles(M, N) ? 127 : 63)) / (big_tiles(M, N) ? 128 : 64); }

int gemm(GemmArgs g, int splits, hipStream_t s);

int gemm(GemmArgs g, int splits, hipStream_t s) {
  if (g.mask && g.N == 256 && g.M >= 128 && splits == 1) {
    // the ReLU backward over all 256 columns in one tile: A (dH2) read once
    dim3 grid(1u, (unsigned)((g.M + 127) / 128), 1u);
    k_gemm<4, 8, true><<<grid, 256, 0, s>>>(g);
  } else if (big_tiles(g.M, g.N) && splits == 1) {
    dim3 grid((unsigned)((g.N + 127) / 128), (unsigned)((g.M + 127) / 128), (unsigned)splits);
    if (g.mask)
      k_gemm<4, 4, true><<<grid, 256, 0, s>>>(g);
    else
      k_gemm<4, 4, false><<<grid, 256, 0, s>>>(g);
  } else if (splits > 1 && g.N >= 128) {
    dim3 grid((unsigned)((g.N + 127) / 128), (unsigned)((g.M + 63) / 64), (unsigned)splits);
    k_gemm<2, 4, false><<<grid, 256, 0, s>>>(g);
  } else {
    dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)splits);
    if (g.mask)
      k_gemm<2, 2, true><<<grid, 256, 0, s>>>(g);
    else
      k_gemm<2, 2, false><<<grid, 256, 0, s>>>(g);
  }
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

// out[i] = sum over splits of part[z * n + i], in split order.
__global__ void k_split_sum(const float *__restrict__ part, int splits, int64_t n,
                            float *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  // eight loads in flight per thread; the sum still runs in split order
#pragma unroll 8
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * n + i];
  out[i] = s;
}

// Weight-gradient partials over one chunk of rows: part[z][i][j] = sum over
// the rows k of chunk z (K steps of 32, ascending) of A[k][i] G[k][j], for
// the whole NA x 256 gradient (A [M][NA], G [M][256], BF16, row-major,
// 16-byte aligned).  One workgroup of 16 waves holds the full gradient, so
// each operand row is read from memory once per product: wave w owns rows
// (w / 4) NA/4 .. and columns (w % 4) 64 .. as (NA/64) x 4 MFMA 16x16x32
// tiles.  A K step's slices of A and G go to LDS transposed ([column][k],
// each k pair one 32-bit word, as the MFMA reads 8 consecutive k per lane);
// the next step's are loaded into registers during this step's MFMAs.  Rows
// at or past the chunk's end (or M) read as zero.
constexpr int kWgThreads = 1024;  // threads per workgroup of k_wgrad
constexpr int kWgRows = 1024;     // fewest rows per chunk (at most 256 chunks)
template <int NA>
__global__ void __launch_bounds__(kWgThreads) k_wgrad(const __bf16 *__restrict__ A,
                                                       const __bf16 *__restrict__ G, int M,
                                                       int kchunk, float *__restrict__ part) {
  constexpr int NB = kHid;
  constexpr int CG = (NA + NB) / 8;     // 8-column groups of both operands
  constexpr int ITEMS = CG * (BK / 2);  // (column group, k pair) staging tasks per K step
  constexpr int TA = NA / 64, TB = 4;
  static_assert(NA % 64 == 0 && ITEMS <= kWgThreads, "k_wgrad shape");
  __shared__ __align__(16) __bf16 T[NA + NB][LDK];  // LDS rows 0..NA-1: A^T; then G^T
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kbeg = blockIdx.x * kchunk, kend = min(M, kbeg + kchunk);
  // this thread's staging task: rows k0 + 2 kp and k0 + 2 kp + 1 of one
  // operand's columns 8 cg' .. 8 cg' + 7
  const bool stager = tid < ITEMS;
  const int kp = tid % (BK / 2), cg = tid / (BK / 2);
  const bool on_a = cg < NA / 8;
  const __bf16 *src = on_a ? A + 8 * cg : G + 8 * (cg - NA / 8);
  const int64_t ld = on_a ? NA : NB;
  bf16x8 lo, hi;
  auto fetch = [&](int k0) {
    const int r = k0 + 2 * kp;
#pragma unroll
    for (int j = 0; j < 8; ++j) lo[j] = hi[j] = (__bf16)0.f;
    if (stager && r < kend) lo = *reinterpret_cast<const bf16x8 *>(src + (int64_t)r * ld);
    if (stager && r + 1 < kend) hi = *reinterpret_cast<const bf16x8 *>(src + (int64_t)(r + 1) * ld);
  };
  const int wr = wave >> 2, wc = wave & 3;
  const int ia = wr * (NA / 4), jb = NA + 64 * wc;  // LDS rows of the wave's A and G tiles
  const int lr = lane & 15, lk = 8 * (lane >> 4);
  f32x4 acc[TA][TB];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();  // every wave has read the previous step's fragments
    if (stager) {
      const u16x8 l = __builtin_bit_cast(u16x8, lo), h = __builtin_bit_cast(u16x8, hi);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        *reinterpret_cast<uint32_t *>(&T[8 * cg + j][2 * kp]) = (uint32_t)l[j] | ((uint32_t)h[j] << 16);
    }
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
    bf16x8 fa[TA], fb[TB];
#pragma unroll
    for (int a = 0; a < TA; ++a) fa[a] = *reinterpret_cast<const bf16x8 *>(&T[ia + 16 * a + lr][lk]);
#pragma unroll
    for (int b = 0; b < TB; ++b) fb[b] = *reinterpret_cast<const bf16x8 *>(&T[jb + 16 * b + lr][lk]);
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
  }
  // the accumulator of tile (a, b) holds rows 4 (lane / 16) .. +3 of column lane % 16
  float *out = part + (int64_t)blockIdx.x * NA * NB;
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(int64_t)(ia + 16 * a + 4 * (lane >> 4) + r) * NB + 64 * wc + 16 * b + lr] = acc[a][b][r];
}

// Column sums over the M rows (bias gradients, the output layer's weight
// gradient) in two deterministic passes: one workgroup per chunk of rows
// writes its partial sums part[chunk][n]; k_col_merge then adds the
// kColChunks partials of each column.  2048 chunks: eight 4-wave workgroups
// per CU, all resident at once (1024 left half the wave slots empty; 4096
// made the merges longer than the pass got shorter).
constexpr int kColChunks = 2048;

// Second pass of the column sums: one workgroup of kMergeThreads per column,
// thread j adds partials j, j + kMergeThreads, ... in order, then each
// wave's lanes combine in a fixed shuffle tree and the waves in order
// (deterministic).
constexpr int kMergeThreads = 256;
__device__ __forceinline__ void col_merge_one(const float *__restrict__ part, int chunks, int N,
                                              int n, float *__restrict__ out) {
  __shared__ float wsum[kMergeThreads / 64];
  const int t = threadIdx.x, lane = t & 63;
  float s = 0.f;
  // four loads in flight per thread; the sum still runs in chunk order
#pragma unroll 4
  for (int z = t; z < chunks; z += kMergeThreads) s += part[(int64_t)z * N + n];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_down(s, d, 64);
  if (lane == 0) wsum[t >> 6] = s;
  __syncthreads();
  if (t == 0) {
    float r = wsum[0];
#pragma unroll
    for (int k = 1; k < kMergeThreads / 64; ++k) r += wsum[k];
    out[n] = r;
  }
}

__global__ void __launch_bounds__(kMergeThreads)
    k_col_merge(const float *__restrict__ part, int chunks, int N, float *__restrict__ out) {
  col_merge_one(part, chunks, N, blockIdx.x, out);
}

// Three column merges in one launch (blocks 0..Na-1: the first array, then
// the second, then the third), each column as k_col_merge sums it.
__global__ void __launch_bounds__(kMergeThreads)
    k_col_merge3(int chunks, const float *__restrict__ pa, int Na, float *__restrict__ oa,
                 const float *__restrict__ pb, int Nb, float *__restrict__ ob,
                 const float *__restrict__ pc, int Nc, float *__restrict__ oc) {
  const int n = blockIdx.x;
  if (n < Na) col_merge_one(pa, chunks, Na, n, oa);
  else if (n < Na + Nb) col_merge_one(pb, chunks, Nb, n - Na, ob);
  else col_merge_one(pc, chunks, Nc, n - Na - Nb, oc);
}


// Output layer (kHid -> kOut = 2) of the forward pass: Y[m] = H2[m] W3 + b3
// with FP32 accumulation.  Half a wave per row: lane l of the half reads
// H2[m][8l .. 8l+7] (16 bytes) and holds W3's rows 8l .. 8l+7; the 32
// partial sums of each output combine in a fixed shuffle tree.
__global__ void __launch_bounds__(256) k_out_forward(const __bf16 *__restrict__ H2,
                                                     const __bf16 *__restrict__ W3,
                                                     const float *__restrict__ b3, int64_t M,
                                                     float *__restrict__ Y) {
  static_assert(kHid == 256 && kOut == 2, "32 lanes of 8 features per row");
  const int lane = threadIdx.x & 63, half = lane >> 5, l = lane & 31;
  float w0[8], w1[8];
  for (int j = 0; j < 8; ++j) {
    w0[j] = (float)W3[(8 * l + j) * kOut];
    w1[j] = (float)W3[(8 * l + j) * kOut + 1];
  }
  const float c0 = b3 ? b3[0] : 0.f, c1 = b3 ? b3[1] : 0.f;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t m0 = 2 * wave; m0 < M; m0 += 2 * nwaves) {
    const int64_t m = m0 + half;
    float s0 = 0.f, s1 = 0.f;
    if (m < M) {
      const bf16x8 h = *reinterpret_cast<const bf16x8 *>(H2 + m * kHid + 8 * l);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        s0 += (float)h[j] * w0[j];
        s1 += (float)h[j] * w1[j];
      }
    }
#pragma unroll
    for (int d = 16; d >= 1; d >>= 1) {
      s0 += __shfl_xor(s0, d, 32);
      s1 += __shfl_xor(s1, d, 32);
    }
    if (l == 0 && m < M) {
      Y[2 * m] = s0 + c0;
      Y[2 * m + 1] = s1 + c1;
    }
  }
}

// The output layer's backward and the second ReLU layer's, in one pass over
// row chunk blockIdx.x of H2 and dY (dY rounded to BF16 for the products):
//   dW3[k][o] = sum_m H2[m][k] dY[m][o] into part3[chunk][2k + o] and
//   db3[o] = sum_m dY[m][o] (FP32) into partb[chunk][o];
//   dH2 = (dY W3^T) * (H2 > 0) in BF16 (the two products added in FP32) and
//   db2's column sums of dH2 into partr[chunk][n].
// k_col_merge adds the chunks.  Wave w takes rows r0 + w, r0 + w + 4, ... in
// order, lane l the features 4l .. 4l+3; the four waves' sums are added in
// wave order.
__global__ void __launch_bounds__(256) k_out_relu_back(const __bf16 *__restrict__ H2,
                                                       const float *__restrict__ dY,
                                                       const __bf16 *__restrict__ W3, int64_t M,
                                                       int64_t chunk, float *__restrict__ part3,
                                                       float *__restrict__ partb,
                                                       __bf16 *__restrict__ G2,
                                                       float *__restrict__ partr) {
  static_assert(kHid == 256 && kOut == 2, "one wave spans a row of 4 x 64 features");
  __shared__ float red[4][64][8];
  __shared__ float4 redr[4][64];
  __shared__ float redb[4][2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(M, r0 + chunk);
  float w3[4][2];
  for (int j = 0; j < 4; ++j) {
    w3[j][0] = (float)W3[(4 * lane + j) * kOut];
    w3[j][1] = (float)W3[(4 * lane + j) * kOut + 1];
  }
  float acc[8];
  for (int i = 0; i < 8; ++i) acc[i] = 0.f;
  float sb0 = 0.f, sb1 = 0.f;
  float sx = 0.f, sy = 0.f, sz = 0.f, sw = 0.f;
  for (int64_t m = r0 + w; m < r1; m += 4) {
    const int64_t i = m * kHid + 4 * lane;
    const float y0 = dY[2 * m], y1 = dY[2 * m + 1];
    const float q0 = (float)(__bf16)y0, q1 = (float)(__bf16)y1;
    const bf16x4 h = *reinterpret_cast<const bf16x4 *>(H2 + i);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[2 * j] += (float)h[j] * q0;
      acc[2 * j + 1] += (float)h[j] * q1;
    }
    sb0 += y0;
    sb1 += y1;
    float4 g;
    g.x = q0 * w3[0][0] + q1 * w3[0][1];
    g.y = q0 * w3[1][0] + q1 * w3[1][1];
    g.z = q0 * w3[2][0] + q1 * w3[2][1];
    g.w = q0 * w3[3][0] + q1 * w3[3][1];
    const float vx = (float)h[0] > 0.f ? g.x : 0.f, vy = (float)h[1] > 0.f ? g.y : 0.f;
    const float vz = (float)h[2] > 0.f ? g.z : 0.f, vw = (float)h[3] > 0.f ? g.w : 0.f;
    sx += vx;
    sy += vy;
    sz += vz;
    sw += vw;
    bf16x4 b;
    b[0] = (__bf16)vx;
    b[1] = (__bf16)vy;
    b[2] = (__bf16)vz;
    b[3] = (__bf16)vw;
    *reinterpret_cast<bf16x4 *>(G2 + i) = b;
  }
  for (int i = 0; i < 8; ++i) red[w][lane][i] = acc[i];
  redr[w][lane] = make_float4(sx, sy, sz, sw);
  if (lane == 0) {
    redb[w][0] = sb0;
    redb[w][1] = sb1;
  }
  __syncthreads();
  if (w == 0) {
    for (int i = 0; i < 8; ++i) {
      float t = red[0][lane][i];
      for (int k = 1; k < 4; ++k) t += red[k][lane][i];
      part3[(int64_t)blockIdx.x * (kHid * kOut) + 8 * lane + i] = t;
    }
    if (lane < kOut) {
      float t = redb[0][lane];
      for (int k = 1; k < 4; ++k) t += redb[k][lane];
      partb[(int64_t)blockIdx.x * kOut + lane] = t;
    }
  } else if (w == 1) {
    float4 t = redr[0][lane];
    for (int k = 1; k < 4; ++k) {
      const float4 u = redr[k][lane];
      t.x += u.x;
      t.y += u.y;
      t.z += u.z;
      t.w += u.w;
    }
    *reinterpret_cast<float4 *>(partr + (int64_t)blockIdx.x * kHid + 4 * lane) = t;
  }
}

// Features of FGT edges (the child node's card state and score), one row of
// 192 BF16 values per edge:
//   0..155   Alex's hand, Bob's hand and the pool as three 52-bit masks;
//   156..159 inherited score: ca/7, cb/7, d/16, +1/-1/0 for the 7-club bonus
//            owner (Alex/Bob/none);
//   160..166 the round so far (the GT node's running score): Alex's and
//            Bob's clubs /13, last picker +1/-1/0 (Alex/Bob/none), Alex's
//            points /10 and Surs, Bob's points /10 and Surs;
//   167..175 one-hot of the node's level (0..8);
//   176..191 zero.
struct HandCards {
  uint8_t card[8];
};

__device__ void feature_row(int32_t q, const int32_t *__restrict__ f_gt,
                            const int32_t *__restrict__ f_sid, const uint64_t *__restrict__ pool,
                            const uint8_t *__restrict__ hands, const int8_t *__restrict__ rs,
                            const int8_t *__restrict__ tab, int level, const HandCards &hc,
                            __bf16 *__restrict__ row) {
  const int32_t g = f_gt[q];
  const uint8_t h = hands[g];
  uint64_t ha = 0, hb = 0;
  for (int b = 0; b < 4; ++b) {
    if ((h >> b) & 1) ha |= 1ull << hc.card[b];
    if ((h >> (4 + b)) & 1) hb |= 1ull << hc.card[4 + b];
  }
  const uint64_t p = pool[g];
  const __bf16 one = (__bf16)1.f, zero = (__bf16)0.f;
  for (int c = 0; c < 52; ++c) {
    row[c] = ((ha >> c) & 1) ? one : zero;
    row[52 + c] = ((hb >> c) & 1) ? one : zero;
    row[104 + c] = ((p >> c) & 1) ? one : zero;
  }
  const int8_t *s = tab + 4 * f_sid[q];
  row[156] = (__bf16)((float)s[0] / 7.f);
  row[157] = (__bf16)((float)s[1] / 7.f);
  row[158] = (__bf16)((float)s[2] / 16.f);
  row[159] = (__bf16)(s[3] == 1 ? 1.f : (s[3] == 2 ? -1.f : 0.f));
  const int8_t *r = rs + 8 * (int64_t)g;  // Acl, Bcl, last picker, Apt, Asr, Bpt, Bsr
  row[160] = (__bf16)((float)r[0] / 13.f);
  row[161] = (__bf16)((float)r[1] / 13.f);
  row[162] = (__bf16)(r[2] == 1 ? 1.f : (r[2] == 2 ? -1.f : 0.f));
  row[163] = (__bf16)((float)r[3] / 10.f);
  row[164] = (__bf16)(float)r[4];
  row[165] = (__bf16)((float)r[5] / 10.f);
  row[166] = (__bf16)(float)r[6];
  for (int c = 167; c < kIn; ++c) row[c] = zero;
  row[167 + level] = one;
}

__global__ void k_features(int64_t n, const int32_t *__restrict__ edges, const int32_t *__restrict__ f_gt,
                           const int32_t *__restrict__ f_sid, const uint64_t *__restrict__ pool,
                           const uint8_t *__restrict__ hands, const int8_t *__restrict__ rs,
                           const int8_t *__restrict__ tab, int level, HandCards hc,
                           __bf16 *__restrict__ X) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  feature_row(edges ? edges[i] : (int32_t)i, f_gt, f_sid, pool, hands, rs, tab, level, hc,
              X + i * kIn);
}

// Feature rows of every node of levels 1..nl, level by level (row off[l-1] +
// q for node q of level l).
struct FeatLevels {
  const int32_t *f_gt[9], *f_sid[9];
  const uint64_t *pool[9];
  const uint8_t *hands[9];
  const int8_t *rs[9];
  int64_t off[9];  // off[l-1] = first row of level l; off[nl] = rows
  int nl;
};

__global__ void k_features_levels(FeatLevels F, const int8_t *__restrict__ tab, HandCards hc,
                                  __bf16 *__restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= F.off[F.nl]) return;
  int l = 1;
  while (l < F.nl && i >= F.off[l]) ++l;
  feature_row((int32_t)(i - F.off[l - 1]), F.f_gt[l], F.f_sid[l], F.pool[l], F.hands[l], F.rs[l],
              tab, l, hc, X + i * kIn);
}

// Policy / value loss gradient.  seg[p]..seg[p+1] are the rows (edges) of
// parent p; Y[r] = (logit, value).  Policy: cross-entropy between the
// softmax of the logits over the siblings and the target strategy, averaged
// over parents; value: vw/2 (value - target)^2 averaged over rows.
__global__ void k_loss(int64_t n_par, const int32_t *__restrict__ seg, const float *__restrict__ Y,
                       const float *__restrict__ tsig, const float *__restrict__ tval, float vw,
                       int64_t n_rows, float *__restrict__ dY, float *__restrict__ loss) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_par) return;
  const int32_t b = seg[p], e = seg[p + 1];
  float mx = -INFINITY;
  for (int32_t r = b; r < e; ++r) mx = fmaxf(mx, Y[2 * r]);
  float z = 0.f;
  for (int32_t r = b; r < e; ++r) z += expf(Y[2 * r] - mx);
  float lp = 0.f, lv = 0.f;
  const float inv_p = 1.f / (float)n_par, inv_r = 1.f / (float)n_rows;
  for (int32_t r = b; r < e; ++r) {
    const float pr = expf(Y[2 * r] - mx) / z;
    dY[2 * r] = (pr - tsig[r]) * inv_p;
    if (tsig[r] > 0.f) lp -= tsig[r] * logf(fmaxf(pr, 1e-30f));
    const float dv = Y[2 * r + 1] - tval[r];
    dY[2 * r + 1] = vw * dv * inv_r;
    lv += 0.5f * vw * dv * dv;
  }
  loss[2 * p] = lp * inv_p;
  loss[2 * p + 1] = lv * inv_r;
}

// One Adam element: moments, master weight and its BF16 copy.
__device__ __forceinline__ void adam_elem(int64_t i, float *__restrict__ w,
                                          const float *__restrict__ g, float *__restrict__ m,
                                          float *__restrict__ v, __bf16 *__restrict__ wb, float lr,
                                          float b1, float b2, float eps, float c1, float c2) {
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = (__bf16)wi;
}

__global__ void k_adam(int64_t n, float *__restrict__ w, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, __bf16 *__restrict__ wb,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  adam_elem(i, w, g, m, v, wb, lr, b1, b2, eps, c1, c2);
}

// Up to kAdamMax arrays in one launch: array t covers flat elements
// off[t] .. off[t+1]-1.
constexpr int kAdamMax = 8;
struct AdamSet {
  int count;
  int64_t off[kAdamMax + 1];
  float *w[kAdamMax];
  const float *g[kAdamMax];
  float *m[kAdamMax];
  float *v[kAdamMax];
  __bf16 *wb[kAdamMax];
};

__global__ void k_adam_multi(AdamSet a, float lr, float b1, float b2, float eps, float c1,
                             float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.off[a.count]) return;
  int t = 0;
  while (t + 1 < a.count && i >= a.off[t + 1]) ++t;
  adam_elem(i - a.off[t], a.w[t], a.g[t], a.m[t], a.v[t], a.wb[t], lr, b1, b2, eps, c1, c2);
}

__global__ void k_sgd(int64_t n, float *__restrict__ w, const float *__restrict__ g,
                      __bf16 *__restrict__ wb, float lr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float wi = w[i] - lr * g[i];
  w[i] = wi;
  if (wb) wb[i] = (__bf16)wi;
}

// Warm start of one level: sigma = softmax of the predicted logits over
// each parent's children; R = kappa_r * sigma; Sbar = kappa_s * sigma.
template <class T>
__global__ void k_warm_init(int64_t np, const int32_t *__restrict__ cb, const float *__restrict__ Y,
                            float kappa_r, float kappa_s, T *__restrict__ sigma, T *__restrict__ R,
                            T *__restrict__ Sbar) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= np) return;
  const int32_t b = cb[h], e = cb[h + 1];
  double mx = -INFINITY;
  for (int32_t q = b; q < e; ++q) mx = fmax(mx, (double)Y[2 * q]);
  double z = 0.0;
  for (int32_t q = b; q < e; ++q) z += exp((double)Y[2 * q] - mx);
  for (int32_t q = b; q < e; ++q) {
    const double s = exp((double)Y[2 * q] - mx) / z;
    sigma[q] = (T)s;
    R[q] = (T)(kappa_r * s);
    Sbar[q] = (T)(kappa_s * s);
  }
}

// The same for the children of every node of levels 0..nl-1 in one launch:
// parent j of level l is node j - poff[l]; its children's logits are rows
// yoff[l] + child index of Y.
template <class T>
struct WarmLevels {
  const int32_t *cb[9];
  T *sigma[9], *R[9], *Sbar[9];  // of the child level l+1
  int64_t poff[9], yoff[9];
  int nl;
};

template <class T>
__global__ void k_warm_init_levels(WarmLevels<T> W, const float *__restrict__ Y, float kappa_r,
                                   float kappa_s) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= W.poff[W.nl]) return;
  int l = 0;
  while (l + 1 < W.nl && j >= W.poff[l + 1]) ++l;
  const int64_t h = j - W.poff[l];
  const int32_t b = W.cb[l][h], e = W.cb[l][h + 1];
  const float *y = Y + 2 * W.yoff[l];
  double mx = -INFINITY;
  for (int32_t q = b; q < e; ++q) mx = fmax(mx, (double)y[2 * q]);
  double z = 0.0;
  for (int32_t q = b; q < e; ++q) z += exp((double)y[2 * q] - mx);
  for (int32_t q = b; q < e; ++q) {
    const double sv = exp((double)y[2 * q] - mx) / z;
    W.sigma[l][q] = (T)sv;
    W.R[l][q] = (T)(kappa_r * sv);
    W.Sbar[l][q] = (T)(kappa_s * sv);
  }
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------------------
// Fused inference: Y = (relu(relu(X W1 + b1) W2 + b2)) W3 + b3 for a tile of
// 128 rows per workgroup, H1 and H2 kept in LDS (rounded to BF16 as in
// pasur_mlp_forward).  The hidden layer overwrites the input tile in place
// (every wave has read the tile when the first hidden values are written),
// so a workgroup holds 70 KB of LDS and two workgroups share a CU: the
// latency of one's tile load and epilogues hides behind the other's MFMAs.
// The MFMA computes each layer transposed, D = W^T A^T:
// the weights (pre-transposed to [out][in], contiguous in K) are the A
// operand, loaded from global memory (L2-resident, shared by all
// workgroups) 16 bytes per lane and prefetched one K step ahead; the
// activations (row-major in LDS, contiguous in K) are the B operand.  A
// 16x16 result tile then holds four consecutive output features of one row
// per lane, which store as one 8-byte LDS write.  With W waves, wave w owns
// output features 256/W consecutive from w*256/W for all 128 rows
// (256/(16W) x 8 tiles of 16x16x32).  The biases and W3 (transposed) are
// staged in LDS with the input tile, so that no epilogue waits on memory.
constexpr int IM = 128;                 // rows per workgroup
constexpr int kInferWaves = 8;          // two waves per SIMD per workgroup, two workgroups per CU
constexpr int kInferDepth = 1;          // K steps of weight fragments in flight per wave
constexpr int XS = kIn + 8, HS = kHid + 8;  // LDS row strides (bf16), 16-byte aligned

// One hidden layer of the fused inference for a wave's 16*TA output features
// and all 16*TB rows: the weight fragments (A operand, from global memory)
// run DEPTH K steps ahead in a ring of registers, so that their L2 latency
// hides behind the MFMAs of the steps in between; activations (B operand)
// come from LDS.  Writes bf16(relu(acc + bias)) into Hs after every wave has
// read As.
template <int K, int TA, int TB, int DEPTH>
__device__ __forceinline__ void infer_layer(const __bf16 *__restrict__ Wt, const __bf16 *As, int as,
                                            const float *__restrict__ bias, __bf16 *Hs, int n_base,
                                            int lane) {
  constexpr int NS = K / 32;
  const int lr = lane & 15, lk = 8 * (lane >> 4);
  f32x4 acc[TA][TB];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ring[DEPTH][TA];
#pragma unroll
  for (int st = 0; st < DEPTH; ++st)
    if (st < NS)
#pragma unroll
      for (int a = 0; a < TA; ++a)
        ring[st][a] = *reinterpret_cast<const bf16x8 *>(Wt + (int64_t)(n_base + 16 * a + lr) * K +
                                                        32 * st + lk);
#pragma unroll
  for (int st = 0; st < NS; ++st) {
    bf16x8 wcur[TA];
#pragma unroll
    for (int a = 0; a < TA; ++a) wcur[a] = ring[st % DEPTH][a];
    if (st + DEPTH < NS) {
#pragma unroll
      for (int a = 0; a < TA; ++a)
        ring[st % DEPTH][a] = *reinterpret_cast<const bf16x8 *>(
            Wt + (int64_t)(n_base + 16 * a + lr) * K + 32 * (st + DEPTH) + lk);
    }
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      const bf16x8 x = *reinterpret_cast<const bf16x8 *>(As + (16 * b + lr) * as + 32 * st + lk);
#pragma unroll
      for (int a = 0; a < TA; ++a)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wcur[a], x, acc[a][b], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave has read As before Hs is (over)written
#pragma unroll
  for (int a = 0; a < TA; ++a) {
    const int n = n_base + 16 * a + 4 * (lane >> 4);
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      const int m = 16 * b + lr;
      typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
      bf16x4 h;
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = (__bf16)fmaxf(acc[a][b][i] + bias[n + i], 0.f);
      *reinterpret_cast<bf16x4 *>(Hs + m * HS + n) = h;
    }
  }
  __syncthreads();
}

// A tile's hidden layer (IM rows of Hs, LDS) to H [M][256] in global memory
// as 16-byte row pieces, rows below M only.
template <int NT>
__device__ __forceinline__ void store_hidden(const __bf16 *Hs, __bf16 *__restrict__ H, int m0,
                                             int M, int tid) {
  for (int e = tid; e < IM * (kHid / 8); e += NT) {
    const int r = e / (kHid / 8), c = (e % (kHid / 8)) * 8;
    if (m0 + r < M)
      *reinterpret_cast<bf16x8 *>(H + (int64_t)(m0 + r) * kHid + c) =
          *reinterpret_cast<const bf16x8 *>(Hs + r * HS + c);
  }
}

// STORE: the training forward pass, which also writes H1 and H2 (for the
// backward pass) from LDS as they are formed.
template <int WAVES, int DEPTH, bool STORE>
__global__ void __launch_bounds__(64 * WAVES) k_mlp_infer(int M, const __bf16 *__restrict__ X,
                                                   const __bf16 *__restrict__ W1t,
                                                   const float *__restrict__ b1,
                                                   const __bf16 *__restrict__ W2t,
                                                   const float *__restrict__ b2,
                                                   const __bf16 *__restrict__ W3,
                                                   const float *__restrict__ b3,
                                                   float *__restrict__ Y, __bf16 *__restrict__ H1,
                                                   __bf16 *__restrict__ H2) {
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16 *Xs = reinterpret_cast<__bf16 *>(smem);          // [IM][XS], the input tile
  __bf16 *Hs = Xs;                                         // [IM][HS], in its place
  float *b1s = reinterpret_cast<float *>(smem + sizeof(__bf16) * IM * HS);  // [kHid]
  float *b2s = b1s + kHid;                                                   // [kHid]
  __bf16 *w3s = reinterpret_cast<__bf16 *>(b2s + kHid);    // [kOut][kHid], W3 transposed
  constexpr int NT = 64 * WAVES;         // threads
  constexpr int TA = kHid / 16 / WAVES;  // 16-wide output tiles per wave
  constexpr int TB = IM / 16;            // 16-row tiles per workgroup
  constexpr int XP = IM * (kIn / 8) / NT;  // 16-byte pieces of the tile per thread
  static_assert(IM * (kIn / 8) % NT == 0 && NT >= kHid, "tile staging");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * IM;
  // X tile, biases and W3 -> LDS: every load issued before the first LDS
  // write (rows past M are zero)
  bf16x8 xv[XP];
#pragma unroll
  for (int i = 0; i < XP; ++i) {
    const int e = tid + i * NT, r = e / (kIn / 8), c = (e % (kIn / 8)) * 8;
    if (m0 + r < M) xv[i] = *reinterpret_cast<const bf16x8 *>(X + (int64_t)(m0 + r) * kIn + c);
    else
#pragma unroll
      for (int j = 0; j < 8; ++j) xv[i][j] = (__bf16)0.f;
  }
  float bv1 = 0.f, bv2 = 0.f;
  __bf16 wv[kOut];
  if (tid < kHid) {
    bv1 = b1[tid];
    bv2 = b2[tid];
#pragma unroll
    for (int o = 0; o < kOut; ++o) wv[o] = W3[tid * kOut + o];
  }
  const float bo0 = b3[0], bo1 = b3[1];
#pragma unroll
  for (int i = 0; i < XP; ++i) {
    const int e = tid + i * NT, r = e / (kIn / 8), c = (e % (kIn / 8)) * 8;
    *reinterpret_cast<bf16x8 *>(Xs + r * XS + c) = xv[i];
  }
  if (tid < kHid) {
    b1s[tid] = bv1;
    b2s[tid] = bv2;
#pragma unroll
    for (int o = 0; o < kOut; ++o) w3s[o * kHid + tid] = wv[o];
  }
  __syncthreads();
  const int n_base = wave * 16 * TA;   // this wave's output features
  infer_layer<kIn, TA, TB, DEPTH>(W1t, Xs, XS, b1s, Hs, n_base, lane);  // H1 in Hs
  // (layer 2 reads Hs and passes a barrier before it overwrites it)
  if (STORE) store_hidden<NT>(Hs, H1, m0, M, tid);
  infer_layer<kHid, TA, TB, DEPTH>(W2t, Hs, HS, b2s, Hs, n_base, lane);  // H2 in Hs
  if (STORE) store_hidden<NT>(Hs, H2, m0, M, tid);
  // last layer (256 -> 2) on the matrix cores as well: wave v < IM/16 takes
  // rows 16v..16v+15; the A operand is W3 transposed and padded to 16
  // outputs (rows 2..15 zero), read from LDS; outputs 0 and 1 of row
  // 16v + (lane & 15) land in elements 0 and 1 of lanes 0..15.
  if (wave < IM / 16) {
    const int lr = lane & 15, lk = 8 * (lane >> 4);
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < kHid; k0 += 32) {
      bf16x8 wa;
      if (lr < kOut) wa = *reinterpret_cast<const bf16x8 *>(w3s + lr * kHid + k0 + lk);
      else
#pragma unroll
        for (int i = 0; i < 8; ++i) wa[i] = (__bf16)0.f;
      const bf16x8 x = *reinterpret_cast<const bf16x8 *>(Hs + (16 * wave + lr) * HS + k0 + lk);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, x, acc, 0, 0, 0);
    }
    const int m = m0 + 16 * wave + lr;
    if (lane < 16 && m < M) {
      Y[(int64_t)m * kOut + 0] = acc[0] + bo0;
      Y[(int64_t)m * kOut + 1] = acc[1] + bo1;
    }
  }
}

static_assert(XS <= HS && kOut == 2, "fused inference layout");
constexpr size_t kInferLds =
    sizeof(__bf16) * (size_t)IM * HS + sizeof(float) * 2 * kHid + sizeof(__bf16) * kOut * kHid;

// W [K][N] (row-major) -> Wt [N][K]
__device__ __forceinline__ void transpose_elem(const __bf16 *__restrict__ W, int K, int N, int i,
                                               __bf16 *__restrict__ Wt) {
  const int k = i / N, n = i % N;
  Wt[(int64_t)n * K + k] = W[i];
}

// W1 [192][256] -> W1t [256][192] and W2 [256][256] -> W2t in one launch
// (elements 0 .. 192*256-1 of the grid: W1, then W2)
__global__ void k_transpose_w12(const __bf16 *__restrict__ W1, __bf16 *__restrict__ W1t,
                                const __bf16 *__restrict__ W2, __bf16 *__restrict__ W2t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kIn * kHid) transpose_elem(W1, kIn, kHid, i, W1t);
  else if (i < kIn * kHid + kHid * kHid) transpose_elem(W2, kHid, kHid, i - kIn * kHid, W2t);
}


template <class T>
__global__ void k_gather(const T *__restrict__ src, const int32_t *__restrict__ idx, int64_t n,
                         float *__restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[idx ? idx[i] : i];
}

__global__ void k_shift(const int32_t *__restrict__ src, int64_t n, int32_t add,
                        int32_t *__restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i] + add;
}

// SplitMix64 finaliser as a hash of (seed, level, parent).
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_sel_flags(int64_t np, const int32_t *__restrict__ cb, uint64_t seed, int level,
                            uint64_t thr, int32_t *__restrict__ flags) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= np) return;
  const bool decision = cb[h + 1] - cb[h] >= 2;
  const uint64_t key = mix64(seed ^ ((uint64_t)level << 56) ^ (uint64_t)h);
  flags[h] = (decision && key <= thr) ? 1 : 0;
}

__global__ void k_sel_compact(int64_t np, const int32_t *__restrict__ flags,
                              const int32_t *__restrict__ pos, const int32_t *__restrict__ cb,
                              int32_t *__restrict__ par, int32_t *__restrict__ fan) {
  int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= np || !flags[h]) return;
  par[pos[h]] = (int32_t)h;
  fan[pos[h]] = cb[h + 1] - cb[h];
}

__global__ void k_sel_expand(int64_t n_sel, const int32_t *__restrict__ par,
                             const int32_t *__restrict__ seg, const int32_t *__restrict__ cb,
                             int32_t *__restrict__ edges) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_sel) return;
  const int32_t h = par[p];
  for (int32_t i = 0; i < seg[p + 1] - seg[p]; ++i) edges[seg[p] + i] = cb[h] + i;
}

}  // namespace

// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------

extern "C" int pasur_gemm_bf16(int M, int N, int K, const uint16_t *A, int64_t sar, int64_t sac,
                               const uint16_t *B, int64_t sbr, int64_t sbc, float *Cf,
                               uint16_t *Cb, int64_t ldc, const float *bias, int relu,
                               void *stream) {
  if (M < 0 || N < 0 || K < 1 || !A || !B || (!Cf && !Cb)) {
    set_error("bad GEMM arguments");
    return PASUR_E_INVAL;
  }
  if (M == 0 || N == 0) return PASUR_OK;
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.M = M; g.N = N; g.K = K;
  g.A = (const __bf16 *)A; g.sar = sar; g.sac = sac;
  g.B = (const __bf16 *)B; g.sbr = sbr; g.sbc = sbc;
  g.Cf = Cf; g.Cb = (__bf16 *)Cb; g.ldc = ldc; g.split_stride = 0;
  g.bias = bias; g.relu = relu; g.kchunk = K;
  return gemm(g, 1, (hipStream_t)stream);
}

namespace {
template <bool STORE>
int fused_forward(const pasur_mlp_weights *w, const uint16_t *X, int64_t M, float *Y, uint16_t *H1,
                  uint16_t *H2, hipStream_t s);
}  // namespace

extern "C" int pasur_mlp_forward(const pasur_mlp_weights *w, const uint16_t *X, int64_t M,
                                 uint16_t *H1, uint16_t *H2, float *Y, void *stream) {
  if (!w || !X || !H1 || !H2 || !Y || M < 0 || M > INT32_MAX) {
    set_error("bad MLP forward arguments");
    return PASUR_E_INVAL;
  }
  if (M == 0) return PASUR_OK;
  hipStream_t s = (hipStream_t)stream;
  if (((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(H1) |
        reinterpret_cast<uintptr_t>(H2)) & 15) == 0)
    // all three layers in the fused kernel, H1 and H2 written from LDS
    return fused_forward<true>(w, X, M, Y, H1, H2, s);
  const int m = (int)M;
  PASUR_TRY(pasur_gemm_bf16(m, kHid, kIn, X, kIn, 1, w->W1, kHid, 1, nullptr, H1, kHid, w->b1, 1, s));
  PASUR_TRY(pasur_gemm_bf16(m, kHid, kHid, H1, kHid, 1, w->W2, kHid, 1, nullptr, H2, kHid, w->b2, 1, s));
  if ((reinterpret_cast<uintptr_t>(H2) & 15) == 0) {
    // the 2-wide output layer as one dot product pair per row (a 64-wide
    // GEMM tile would be 97% padding)
    // 8 rows per workgroup and pass, at most 2048 workgroups (grid-stride)
    const unsigned grid = (unsigned)std::min<int64_t>(2048, (M + 7) / 8);
    k_out_forward<<<grid, 256, 0, s>>>((const __bf16 *)H2, (const __bf16 *)w->W3, w->b3, M, Y);
    PASUR_TRY_HIP(hipGetLastError());
  } else {
    PASUR_TRY(pasur_gemm_bf16(m, kOut, kHid, H2, kHid, 1, w->W3, kOut, 1, Y, nullptr, kOut, w->b3, 0, s));
  }
  return PASUR_OK;
}

namespace {
// The backward pass's workspace, kept per (device, stream) between calls:
// stream order finishes one call's use before the next call's kernels run,
// and a kept block spares every call the stream-ordered allocation and free
// (each of which holds up the queue).  Grown stream-ordered when a call
// needs more; held until the process ends.
std::mutex g_bwd_mu;
std::map<std::pair<int, hipStream_t>, std::pair<void *, size_t>> g_bwd_ws;

int backward_workspace(hipStream_t s, size_t bytes, void **out) {
  int dev = 0;
  PASUR_TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_bwd_mu);
  std::pair<void *, size_t> &ws = g_bwd_ws[std::make_pair(dev, s)];
  if (ws.second < bytes) {
    if (ws.first) (void)hipFreeAsync(ws.first, s);
    ws = std::make_pair(nullptr, (size_t)0);
    void *p = nullptr;
    const hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess) {
      set_error("MLP backward workspace (%zu bytes): %s", bytes, hipGetErrorString(e));
      return PASUR_E_NOMEM;
    }
    ws = std::make_pair(p, bytes);
  }
  *out = ws.first;
  return PASUR_OK;
}
}  // namespace

extern "C" int pasur_mlp_backward(const pasur_mlp_weights *w, const uint16_t *X,
                                  const uint16_t *H1, const uint16_t *H2, const float *dY,
                                  int64_t M, pasur_mlp_grads *gr, void *stream) {
  if (!w || !X || !H1 || !H2 || !dY || !gr || M < 1 || M > INT32_MAX) {
    set_error("bad MLP backward arguments");
    return PASUR_E_INVAL;
  }
  if ((reinterpret_cast<uintptr_t>(H1) & 7) || (reinterpret_cast<uintptr_t>(H2) & 7)) {
    set_error("H1 and H2 must be 8-byte aligned");
    return PASUR_E_INVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int m = (int)M;
  // workspace: dH in BF16 for both hidden layers, split-K and row-chunk
  // partials.  Weight gradients reduce over the M rows in chunks of at least
  // 2048 rows, up to 128 chunks.
  const int splits = std::min(128, std::max(1, m / 2048));
  const int kchunk = ((m + splits - 1) / splits + BK - 1) / BK * BK;
  // k_wgrad's chunks (16-byte aligned operands): up to 256 of at least
  // kWgRows rows each, a multiple of BK
  const int64_t wsplits0 = std::min<int64_t>(256, (M + kWgRows - 1) / kWgRows);
  const int wchunk = (int)(((M + wsplits0 - 1) / wsplits0 + BK - 1) / BK * BK);
  const int wsplits = (int)((M + wchunk - 1) / wchunk);
  // split-K partials of the weight gradients, or the row-chunk partials of
  // the bias gradients and of the output layer's weight gradient, or the
  // dH1 product's row-tile partials of db1
  const size_t part_n = std::max({(size_t)std::max(splits, wsplits) * kHid * kHid,
                                  (size_t)kColChunks * (kHid * kOut + kOut + kHid),
                                  (size_t)row_tiles(m, kHid) * kHid});
  // workspace: dH2 and dH1 in BF16, then the partials
  const size_t gbytes = align_up(sizeof(__bf16) * (size_t)m * kHid, 256);
  void *ws = nullptr;
  PASUR_TRY(backward_workspace(s, 2 * gbytes + sizeof(float) * part_n, &ws));
  __bf16 *G2b = reinterpret_cast<__bf16 *>(ws);
  __bf16 *G1b = reinterpret_cast<__bf16 *>(reinterpret_cast<char *>(ws) + gbytes);
  float *part = reinterpret_cast<float *>(reinterpret_cast<char *>(ws) + 2 * gbytes);
  hipError_t e = hipSuccess;
  int st = PASUR_OK;
  auto dW = [&](const __bf16 *Act, int kin, const __bf16 *G, int nout, float *out) -> int {
    // out[kin, nout] = Act^T G, reduced over the M rows in chunks
    if (nout == kHid && (kin == kHid || kin == kIn) &&
        ((reinterpret_cast<uintptr_t>(Act) | reinterpret_cast<uintptr_t>(G)) & 15) == 0) {
      if (kin == kHid) k_wgrad<kHid><<<wsplits, kWgThreads, 0, s>>>(Act, G, m, wchunk, part);
      else k_wgrad<kIn><<<wsplits, kWgThreads, 0, s>>>(Act, G, m, wchunk, part);
      PASUR_TRY_HIP(hipGetLastError());
      k_split_sum<<<blocks((int64_t)kin * nout, 64), 64, 0, s>>>(part, wsplits, (int64_t)kin * nout, out);
      PASUR_TRY_HIP(hipGetLastError());
      return PASUR_OK;
    }
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.M = kin; g.N = nout; g.K = m;
    g.A = Act; g.sar = 1; g.sac = kin;
    g.B = G; g.sbr = nout; g.sbc = 1;
    g.Cf = part; g.ldc = nout; g.split_stride = (int64_t)kin * nout;
    g.kchunk = kchunk;
    int r = gemm(g, splits, s);
    if (r) return r;
    // 64-thread workgroups: 1024 of them for a 256x256 gradient, every CU busy
    k_split_sum<<<blocks((int64_t)kin * nout, 64), 64, 0, s>>>(part, splits, (int64_t)kin * nout, out);
    return PASUR_OK;
  };
  const int64_t rchunk = (M + kColChunks - 1) / kColChunks;
  if (!st) {
    // layer 3: dW3 = H2^T dY, db3 = colsum dY; dH2 = (dY W3^T) masked by
    // H2 > 0, in BF16, and db2 = its column sums (one pass over the rows)
    float *part3 = part, *partb = part + (size_t)kColChunks * kHid * kOut;
    float *partr = partb + (size_t)kColChunks * kOut;
    k_out_relu_back<<<kColChunks, 256, 0, s>>>((const __bf16 *)H2, dY, (const __bf16 *)w->W3, M,
                                               rchunk, part3, partb, G2b, partr);
    k_col_merge3<<<kHid * kOut + kOut + kHid, kMergeThreads, 0, s>>>(
        kColChunks, part3, kHid * kOut, gr->dW3, partb, kOut, gr->db3, partr, kHid, gr->db2);
    st = dW((const __bf16 *)H1, kHid, G2b, kHid, gr->dW2);
  }
  if (!st) {
    // dH1 = (dH2 W2^T) masked by H1 > 0, in BF16, with db1's row-tile
    // partial sums from the GEMM's epilogue
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.M = m; g.N = kHid; g.K = kHid;
    g.A = G2b; g.sar = kHid; g.sac = 1;
    g.B = (const __bf16 *)w->W2; g.sbr = 1; g.sbc = kHid;  // W2^T
    g.Cb = G1b; g.ldc = kHid; g.kchunk = kHid;
    g.mask = (const __bf16 *)H1; g.colpart = part;
    st = gemm(g, 1, s);
    if (!st) {
      k_col_merge<<<kHid, kMergeThreads, 0, s>>>(part, row_tiles(m, kHid), kHid, gr->db1);
      st = dW((const __bf16 *)X, kIn, G1b, kHid, gr->dW1);
    }
  }
  if (!st) {
    e = hipGetLastError();
    if (e != hipSuccess) {
      set_error("MLP backward: %s", hipGetErrorString(e));
      st = PASUR_E_HIP;
    }
  }
  return st;
}

extern "C" int pasur_mlp_loss(const float *Y, const float *target_sigma, const float *target_value,
                              const int32_t *seg, int64_t n_parents, int64_t n_rows,
                              float value_weight, float *dY, float *loss, void *stream) {
  if (!Y || !target_sigma || !target_value || !seg || !dY || !loss || n_parents < 1 || n_rows < 1) {
    set_error("bad loss arguments");
    return PASUR_E_INVAL;
  }
  k_loss<<<blocks(n_parents), 256, 0, (hipStream_t)stream>>>(n_parents, seg, Y, target_sigma,
                                                             target_value, value_weight, n_rows,
                                                             dY, loss);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_adam_step(float *w, const float *g, float *m, float *v, uint16_t *w_bf16,
                               int64_t n, float lr, float beta1, float beta2, float eps,
                               int64_t step, void *stream) {
  if (!w || !g || !m || !v || n < 0 || step < 1) {
    set_error("bad Adam arguments");
    return PASUR_E_INVAL;
  }
  const float c1 = 1.f - std::pow(beta1, (float)step);
  const float c2 = 1.f - std::pow(beta2, (float)step);
  k_adam<<<blocks(n), 256, 0, (hipStream_t)stream>>>(n, w, g, m, v, (__bf16 *)w_bf16, lr, beta1,
                                                     beta2, eps, c1, c2);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_adam_step_multi(int count, float *const w[], const float *const g[],
                                     float *const m[], float *const v[], uint16_t *const w_bf16[],
                                     const int64_t n[], float lr, float beta1, float beta2,
                                     float eps, int64_t step, void *stream) {
  if (count < 1 || count > kAdamMax || !w || !g || !m || !v || !n || step < 1) {
    set_error("bad multi-array Adam arguments (1..%d arrays)", kAdamMax);
    return PASUR_E_INVAL;
  }
  AdamSet a;
  std::memset(&a, 0, sizeof(a));
  a.count = count;
  for (int t = 0; t < count; ++t) {
    if (!w[t] || !g[t] || !m[t] || !v[t] || n[t] < 0) {
      set_error("bad Adam array %d", t);
      return PASUR_E_INVAL;
    }
    a.off[t + 1] = a.off[t] + n[t];
    a.w[t] = w[t];
    a.g[t] = g[t];
    a.m[t] = m[t];
    a.v[t] = v[t];
    a.wb[t] = w_bf16 ? (__bf16 *)w_bf16[t] : nullptr;
  }
  if (a.off[count] == 0) return PASUR_OK;
  const float c1 = 1.f - std::pow(beta1, (float)step);
  const float c2 = 1.f - std::pow(beta2, (float)step);
  k_adam_multi<<<blocks(a.off[count]), 256, 0, (hipStream_t)stream>>>(a, lr, beta1, beta2, eps, c1,
                                                                        c2);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_sgd_step(float *w, const float *g, uint16_t *w_bf16, int64_t n, float lr,
                              void *stream) {
  if (!w || !g || n < 0) {
    set_error("bad SGD arguments");
    return PASUR_E_INVAL;
  }
  if (n == 0) return PASUR_OK;
  k_sgd<<<blocks(n), 256, 0, (hipStream_t)stream>>>(n, w, g, (__bf16 *)w_bf16, lr);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_edge_features(const pasur_gt *gt, const pasur_fgt *fgt, int level,
                                   const int32_t *d_edges, int64_t n, uint16_t *d_X,
                                   void *stream) {
  if (!gt || !fgt || !d_X || n < 0) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (level < 0 || level > 8) {
    set_error("level %d outside 0..8", level);
    return PASUR_E_RANGE;
  }
  if (!d_edges && n != fgt->n[level]) {
    set_error("without an edge list n must be the level size");
    return PASUR_E_INVAL;
  }
  if (gt->n[0] == 0 || fgt->round != gt->round) {
    set_error("the game tree does not belong to this unfolded tree");
    return PASUR_E_INVAL;
  }
  HandCards hc;
  for (int b = 0; b < 8; ++b) hc.card[b] = gt->deck[4 + 8 * gt->round + b];
  k_features<<<blocks(n), 256, 0, (hipStream_t)stream>>>(
      n, d_edges, fgt->gt[level], fgt->sid[level], gt->pool[level], gt->hands[level],
      (const int8_t *)gt->rs[level], fgt->score_tab, level, hc, (__bf16 *)d_X);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_cfr_warm_init(const pasur_fgt *f, const pasur_cfr_state *st, int level,
                                   const float *Y, float kappa_r, float kappa_s, void *stream) {
  if (!f || !st || !Y) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (level < 1 || level > 8) {
    set_error("level %d outside 1..8", level);
    return PASUR_E_RANGE;
  }
  hipStream_t s = (hipStream_t)stream;
  const int64_t np = f->n[level - 1];
  if (st->dtype == PASUR_F32)
    k_warm_init<float><<<blocks(np), 256, 0, s>>>(np, f->child_begin[level - 1], Y, kappa_r,
                                                  kappa_s, (float *)st->sigma[level],
                                                  (float *)st->R[level], (float *)st->Sbar[level]);
  else
    k_warm_init<double><<<blocks(np), 256, 0, s>>>(np, f->child_begin[level - 1], Y, kappa_r,
                                                   kappa_s, (double *)st->sigma[level],
                                                   (double *)st->R[level], (double *)st->Sbar[level]);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_sample_parents(const pasur_fgt *f, int level, uint64_t seed, double keep_prob,
                                    int32_t *d_seg, int32_t *d_edges, int64_t *n_parents,
                                    int64_t *n_edges, void *stream) {
  if (!f || !d_seg || !d_edges || !n_parents || !n_edges) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (level < 1 || level > 8 || !(keep_prob >= 0.0 && keep_prob <= 1.0)) {
    set_error("need level in 1..8 and keep_prob in [0, 1]");
    return PASUR_E_RANGE;
  }
  hipStream_t s = (hipStream_t)stream;
  const int64_t np = f->n[level - 1];
  const uint64_t thr = keep_prob >= 1.0 ? ~0ull : (uint64_t)(keep_prob * 18446744073709551615.0);
  int32_t *flags = nullptr, *pos = nullptr, *par = nullptr, *fan = nullptr;
  int st = dev_alloc(&flags, np);
  if (!st) st = dev_alloc(&pos, np + 1);
  if (!st) st = dev_alloc(&par, np);
  if (!st) st = dev_alloc(&fan, np);
  int64_t nsel = 0, ne = 0;
  if (!st) {
    k_sel_flags<<<blocks(np), 256, 0, s>>>(np, f->child_begin[level - 1], seed, level, thr, flags);
    st = scan_counts(flags, np, pos, &nsel, s);
  }
  if (!st && nsel > 0) {
    k_sel_compact<<<blocks(np), 256, 0, s>>>(np, flags, pos, f->child_begin[level - 1], par, fan);
    st = scan_counts(fan, nsel, d_seg, &ne, s);
    if (!st) {
      k_sel_expand<<<blocks(nsel), 256, 0, s>>>(nsel, par, d_seg, f->child_begin[level - 1], d_edges);
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        set_error("sample parents: %s", hipGetErrorString(e));
        st = PASUR_E_HIP;
      }
    }
  }
  dev_free(flags);
  dev_free(pos);
  dev_free(par);
  dev_free(fan);
  *n_parents = nsel;
  *n_edges = ne;
  return st;
}

extern "C" int pasur_gather_f32(const void *src, int dtype, const int32_t *idx, int64_t n,
                                float *dst, void *stream) {
  if (!src || !dst || n < 0 || (dtype != PASUR_F32 && dtype != PASUR_F64)) {
    set_error("bad gather arguments");
    return PASUR_E_INVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  if (dtype == PASUR_F32)
    k_gather<float><<<blocks(n), 256, 0, s>>>((const float *)src, idx, n, dst);
  else
    k_gather<double><<<blocks(n), 256, 0, s>>>((const double *)src, idx, n, dst);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

extern "C" int pasur_shift_i32(const int32_t *src, int64_t n, int32_t add, int32_t *dst,
                               void *stream) {
  if (!src || !dst || n < 0) {
    set_error("bad shift arguments");
    return PASUR_E_INVAL;
  }
  k_shift<<<blocks(n), 256, 0, (hipStream_t)stream>>>(src, n, add, dst);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

namespace {
int64_t warm_rows(const pasur_fgt *fgt, int max_level) {
  int64_t rows = 0;
  for (int l = 1; l <= max_level; ++l) rows += fgt->n[l];
  return rows;
}
int64_t warm_bytes(int64_t rows) {
  return (int64_t)align_up((size_t)rows * kIn * sizeof(__bf16), 256) +
         (int64_t)align_up((size_t)rows * kOut * sizeof(float), 256);
}
}  // namespace

extern "C" int64_t pasur_warm_start_workspace_bytes(const pasur_fgt *fgt, int max_level) {
  if (!fgt || max_level < 1 || max_level > 8) return -1;
  return warm_bytes(warm_rows(fgt, max_level));
}

extern "C" int pasur_warm_start_round(const pasur_gt *gt, const pasur_fgt *fgt,
                                      const pasur_cfr_state *st, const pasur_mlp_weights *w,
                                      int max_level, float kappa_r, float kappa_s,
                                      void *workspace, int64_t workspace_bytes, void *stream) {
  if (!gt || !fgt || !st || !w) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  if (max_level < 1 || max_level > 8) {
    set_error("max_level %d outside 1..8", max_level);
    return PASUR_E_RANGE;
  }
  if (gt->n[0] == 0 || fgt->round != gt->round) {
    set_error("the game tree does not belong to this unfolded tree");
    return PASUR_E_INVAL;
  }
  if (st->dtype != PASUR_F32 && st->dtype != PASUR_F64) {
    set_error("unknown dtype %d", st->dtype);
    return PASUR_E_RANGE;
  }
  hipStream_t s = (hipStream_t)stream;
  FeatLevels F;
  std::memset(&F, 0, sizeof(F));
  F.nl = max_level;
  int64_t rows = 0;
  for (int l = 1; l <= max_level; ++l) {
    F.off[l - 1] = rows;
    F.f_gt[l] = fgt->gt[l];
    F.f_sid[l] = fgt->sid[l];
    F.pool[l] = gt->pool[l];
    F.hands[l] = gt->hands[l];
    F.rs[l] = (const int8_t *)gt->rs[l];
    rows += fgt->n[l];
  }
  F.off[max_level] = rows;
  if (rows == 0) return PASUR_OK;
  if (rows > INT32_MAX) {
    set_error("too many rows for one forward pass");
    return PASUR_E_RANGE;
  }
  HandCards hc;
  for (int b = 0; b < 8; ++b) hc.card[b] = gt->deck[4 + 8 * gt->round + b];
  __bf16 *X = nullptr;
  float *Y = nullptr;
  const bool own = !workspace || workspace_bytes < warm_bytes(rows);
  hipError_t e = hipSuccess;
  if (own) {
    e = hipMallocAsync((void **)&X, sizeof(__bf16) * (size_t)rows * kIn, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&Y, sizeof(float) * (size_t)rows * kOut, s);
  } else {
    X = (__bf16 *)workspace;
    Y = (float *)((char *)workspace + align_up((size_t)rows * kIn * sizeof(__bf16), 256));
  }
  int rc = PASUR_OK;
  if (e != hipSuccess) {
    set_error("warm start workspace: %s", hipGetErrorString(e));
    rc = PASUR_E_NOMEM;
  }
  if (!rc) {
    k_features_levels<<<blocks(rows), 256, 0, s>>>(F, fgt->score_tab, hc, X);
    rc = pasur_mlp_infer(w, (const uint16_t *)X, rows, Y, s);
  }
  if (!rc) {
    auto launch = [&](auto *tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      WarmLevels<T> W;
      std::memset(&W, 0, sizeof(W));
      W.nl = max_level;
      int64_t p = 0;
      for (int l = 0; l < max_level; ++l) {
        W.cb[l] = fgt->child_begin[l];
        W.sigma[l] = (T *)st->sigma[l + 1];
        W.R[l] = (T *)st->R[l + 1];
        W.Sbar[l] = (T *)st->Sbar[l + 1];
        W.poff[l] = p;
        W.yoff[l] = F.off[l];
        p += fgt->n[l];
      }
      W.poff[max_level] = p;
      k_warm_init_levels<T><<<blocks(p), 256, 0, s>>>(W, Y, kappa_r, kappa_s);
    };
    if (st->dtype == PASUR_F32) launch((float *)nullptr);
    else launch((double *)nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) {
      set_error("warm start: %s", hipGetErrorString(e));
      rc = PASUR_E_HIP;
    }
  }
  if (own) {
    (void)hipFreeAsync(X, s);
    (void)hipFreeAsync(Y, s);
  }
  return rc;
}

extern "C" int pasur_mlp_transpose(const pasur_mlp_weights *w, uint16_t *W1t, uint16_t *W2t,
                                   void *stream) {
  if (!w || !w->W1 || !w->W2 || !W1t || !W2t) {
    set_error("null argument");
    return PASUR_E_INVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  k_transpose_w12<<<blocks(kIn * kHid + kHid * kHid), 256, 0, s>>>(
      (const __bf16 *)w->W1, (__bf16 *)W1t, (const __bf16 *)w->W2, (__bf16 *)W2t);
  PASUR_TRY_HIP(hipGetLastError());
  return PASUR_OK;
}

namespace {

// The fused kernel over M > 0 rows (inference, or with STORE the training
// forward that also writes H1 and H2): transposed weights from the caller's
// cache, else transposed here into stream-ordered scratch.
template <bool STORE>
int fused_forward(const pasur_mlp_weights *w, const uint16_t *X, int64_t M, float *Y, uint16_t *H1,
                  uint16_t *H2, hipStream_t s) {
  auto kern = k_mlp_infer<kInferWaves, kInferDepth, STORE>;
  // the kernel's LDS exceeds the default limit: raise it once per device
  static std::once_flag lds_once[kMaxDevices];
  static hipError_t lds_err[kMaxDevices];
  int dev = 0;
  PASUR_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the supported %d", dev, kMaxDevices);
    return PASUR_E_RANGE;
  }
  std::call_once(lds_once[dev], [&] {
    lds_err[dev] = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kInferLds);
  });
  if (lds_err[dev] != hipSuccess) {
    set_error("MLP fused forward LDS: %s", hipGetErrorString(lds_err[dev]));
    return PASUR_E_HIP;
  }
  __bf16 *Wt = nullptr;
  const __bf16 *W1t = (const __bf16 *)w->W1t, *W2t = (const __bf16 *)w->W2t;
  hipError_t e = hipSuccess;
  if (!W1t || !W2t) {
    e = hipMallocAsync((void **)&Wt, sizeof(__bf16) * (size_t)(kIn + kHid) * kHid, s);
    if (e != hipSuccess) {
      set_error("MLP fused forward workspace: %s", hipGetErrorString(e));
      return PASUR_E_NOMEM;
    }
    W1t = Wt;
    W2t = Wt + (size_t)kIn * kHid;
    k_transpose_w12<<<blocks(kIn * kHid + kHid * kHid), 256, 0, s>>>(
        (const __bf16 *)w->W1, Wt, (const __bf16 *)w->W2, Wt + (size_t)kIn * kHid);
  }
  kern<<<(unsigned)((M + IM - 1) / IM), 64 * kInferWaves, kInferLds, s>>>(
      (int)M, (const __bf16 *)X, W1t, w->b1, W2t, w->b2, (const __bf16 *)w->W3, w->b3, Y,
      (__bf16 *)H1, (__bf16 *)H2);
  e = hipGetLastError();
  if (Wt) (void)hipFreeAsync(Wt, s);
  if (e != hipSuccess) {
    set_error("MLP fused forward: %s", hipGetErrorString(e));
    return PASUR_E_HIP;
  }
  return PASUR_OK;
}

}  // namespace

extern "C" int pasur_mlp_infer(const pasur_mlp_weights *w, const uint16_t *X, int64_t M,
                               float *Y, void *stream) {
  if (!w || !X || !Y || M < 0 || M > INT32_MAX) {
    set_error("bad MLP inference arguments");
    return PASUR_E_INVAL;
  }
  if (M == 0) return PASUR_OK;
  return fused_forward<false>(w, X, M, Y, nullptr, nullptr, (hipStream_t)stream);
}
