// dm_mlp.hip -- learned warm start of the Newton solve: a 26-256-256-3 ReLU network whose
// matrix products run on the matrix cores in bfloat16 with float32 accumulation
// (v_mfma_f32_16x16x32_bf16), its training (loss, backward pass, Adam), and the per-node
// features and displacement prediction of the implicit step.
//
// Matrix layout: every GEMM operand is stored with its reduction index contiguous, so both
// MFMA operands are 16-byte loads: activations row-major [rows][K] for the batch-row products
// and transposed [K][rows] for the weight gradients, whose reduction runs over the batch.
// Rounding points: every GEMM input is rounded to bfloat16 (nearest, ties to even); biases,
// accumulators, master weights and Adam moments are float32.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <mutex>
#include <stdint.h>
#include <string>
#include <vector>

#define DM_KERNEL_TU
#include "dm_layout.h"
#include "dm_bf16.h"
#include "dmrod.h"

typedef dm_bf16x8 bf16x8;
typedef dm_f32x4 f32x4;
typedef uint16_t u16;

namespace {

constexpr int NI = DM_NET_IN, NH = DM_NET_HID, NO = DM_NET_OUT;
constexpr int KX = DM_NET_KX;             // input width padded to one MFMA reduction step
constexpr int NOP = DM_NET_OUTP;          // output width padded to one MFMA tile
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH, NPARAM = OFF_B3 + NO;
constexpr int ROWS_PAD = 64;              // batch rows are padded to a multiple of this
constexpr int NS_MAX = 64;                // most splits of the weight-gradient batch reduction
constexpr int WG_WAVES = 2048;            // wavefronts aimed at per weight-gradient launch (8 per CU)

__device__ __forceinline__ u16 bf16_bits(float v) { return dm_bf16_bits(v); }
__device__ __forceinline__ float bf16_val(u16 h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) { return dm_mfma_bf16(a, b, c); }
__device__ __forceinline__ bf16x8 ld8(const u16* p) { return *reinterpret_cast<const bf16x8*>(p); }

enum { EPI_HIDDEN = 0, EPI_OUTPUT = 1, EPI_DGRAD = 2 };

// Wavefronts of a row-GEMM workgroup that share one 16-row block, each taking a quarter of the
// column tiles (four when N has at least four tiles, else one wavefront per block).
template <int N>
constexpr int row_wpr() { return N / 16 >= 4 ? 4 : 1; }

// 16-row blocks per wavefront: two where the column tiles are shared out and the reduction is
// long (K >= 64), so each weight fragment loaded serves two MFMAs (half the re-reads of the
// weights over the batch); for K = 32 the weights are small and the wavefronts count more.
template <int K, int N>
constexpr int row_rb() { return row_wpr<N>() == 4 && K >= 64 ? 2 : 1; }

// Workgroups of 256 threads covering `rows` (a multiple of ROWS_PAD) for a K x N product.
template <int K, int N>
inline int row_grid(int rows) { return rows / (16 * row_rb<K, N>() * (4 / row_wpr<N>())); }

// out = epilogue(A[rows][K] . Bm[N][K]^T).  A wavefront computes row_rb 16-row blocks over
// N / 16 / row_wpr column tiles; lane l supplies A[l % 16][8 (l / 16) + 0..7] and, per
// 16-column tile t, Bm[16 t + l % 16][8 (l / 16) + 0..7], and receives
// C[4 (l / 16) + j][16 t + l % 16], j = 0..3.
//   EPI_HIDDEN: + bias, ReLU, bfloat16 to out [rows][N] and outT [N][rows];
//   EPI_OUTPUT: + bias, float32 to outF [rows][3] (columns 0..2);
//   EPI_DGRAD : times the ReLU mask (mask [rows][N] > 0), bfloat16 to out (if given) and outT.
template <int K, int N, int EPI>
__global__ void __launch_bounds__(256) row_gemm(const u16* __restrict__ A, const u16* __restrict__ Bm,
                                                const float* __restrict__ bias, const u16* __restrict__ mask,
                                                int rows, u16* __restrict__ out, u16* __restrict__ outT,
                                                float* __restrict__ outF) {
  constexpr int WPR = row_wpr<N>(), RB = row_rb<K, N>(), TPW = N / 16 / WPR;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row0 = (blockIdx.x * (4 / WPR) + w / WPR) * 16 * RB;
  const int tb = (w % WPR) * TPW;
  if (row0 >= rows) return;
  const int lr = l & 15, lk = 8 * (l >> 4);
  f32x4 acc[RB][TPW];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[b][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) a[b] = ld8(A + (size_t)(row0 + 16 * b + lr) * K + k0 + lk);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const bf16x8 wt = ld8(Bm + (size_t)(16 * (tb + t) + lr) * K + k0 + lk);
#pragma unroll
      for (int b = 0; b < RB; ++b) acc[b][t] = mfma(a[b], wt, acc[b][t]);
    }
  }
#pragma unroll
  for (int rb = 0; rb < RB * TPW; ++rb) {
    const int b = rb / TPW, t = rb % TPW;
    const int r0 = row0 + 16 * b + 4 * (l >> 4);
    const int n = 16 * (tb + t) + lr;
    if (EPI == EPI_OUTPUT) {
      if (n < NO)
#pragma unroll
        for (int j = 0; j < 4; ++j) outF[(size_t)(r0 + j) * NO + n] = acc[b][t][j] + bias[n];
    } else {
      u16 h[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float v = acc[b][t][j];
        if (EPI == EPI_HIDDEN) v = fmaxf(v + bias[n], 0.0f);
        else {
          const u16 m = mask[(size_t)(r0 + j) * N + n];
          v = (m != 0 && !(m & 0x8000)) ? v : 0.0f;
        }
        h[j] = bf16_bits(v);
        if (out) out[(size_t)(r0 + j) * N + n] = h[j];
      }
      uint2 pk;
      pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
      pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
      *reinterpret_cast<uint2*>(outT + (size_t)n * rows + r0) = pk;
    }
  }
}

// Split of the batch reduction of a weight-gradient product with `tiles` output blocks: about
// WG_WAVES wavefronts in all, at most NS_MAX splits, each split a multiple of 32 rows (one
// MFMA reduction step).  ns <= want follows from chunk >= rows / want.
inline void split_plan(int rows, int tiles, int* chunk, int* ns) {
  const int want = std::min(NS_MAX, std::max(1, WG_WAVES / tiles));
  *chunk = ((rows + want - 1) / want + 31) / 32 * 32;
  *ns = (rows + *chunk - 1) / *chunk;
}

// Partial weight gradients over one split of the batch: part[s][m][n] = sum_k At[m][k] Bt[n][k]
// over k in split s (rows s * chunk .. min((s + 1) * chunk, ld) - 1), and (for the first
// column block) bpart[s][m] = sum_k At[m][k].  One wavefront per 16 x NT output block `tile`.
template <int M, int N>
__device__ __forceinline__ void wgrad_block(const u16* __restrict__ At, const u16* __restrict__ Bt, int ld, int chunk,
                                            int tile, int s, float* __restrict__ part, float* __restrict__ bpart) {
  constexpr int NT = N < 64 ? N : 64;
  const int l = threadIdx.x;
  const int mt = tile / (N / NT), nt = tile % (N / NT);
  const int m0 = 16 * mt, n0 = NT * nt;
  const int kb = s * chunk, ke = min(kb + chunk, ld);
  const int lr = l & 15, lk = 8 * (l >> 4);
  f32x4 acc[NT / 16];
#pragma unroll
  for (int t = 0; t < NT / 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bs = 0.0f;
#pragma unroll 4
  for (int k0 = kb; k0 < ke; k0 += 32) {
    const bf16x8 a = ld8(At + (size_t)(m0 + lr) * ld + k0 + lk);
    if (nt == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) bs += (float)a[j];
    }
#pragma unroll
    for (int t = 0; t < NT / 16; ++t) acc[t] = mfma(a, ld8(Bt + (size_t)(n0 + 16 * t + lr) * ld + k0 + lk), acc[t]);
  }
  float* P = part + (size_t)s * M * N;
#pragma unroll
  for (int t = 0; t < NT / 16; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) P[(size_t)(m0 + 4 * (l >> 4) + j) * N + n0 + 16 * t + lr] = acc[t][j];
  if (nt == 0) {
    bs += __shfl_xor(bs, 16, 64);
    bs += __shfl_xor(bs, 32, 64);
    if (l < 16) bpart[(size_t)s * M + m0 + l] = bs;
  }
}

// The three weight-gradient products of one backward pass in one launch.  Product p has
// tiles[p] output blocks and ns[p] splits of chunk[p] rows; its blocks are numbered
// (split, tile) after those of the products before it.
struct WgradSet {
  const u16* At[3];
  const u16* Bt[3];
  float* part[3];
  float* bpart[3];
  int chunk[3], tiles[3], ns[3];
};

__global__ void __launch_bounds__(64) wgrad_all(WgradSet w, int ld) {
  int b = blockIdx.x;
  if (b < w.tiles[0] * w.ns[0]) {
    wgrad_block<NH, NH>(w.At[0], w.Bt[0], ld, w.chunk[0], b % w.tiles[0], b / w.tiles[0], w.part[0], w.bpart[0]);
    return;
  }
  b -= w.tiles[0] * w.ns[0];
  if (b < w.tiles[1] * w.ns[1]) {
    wgrad_block<NH, KX>(w.At[1], w.Bt[1], ld, w.chunk[1], b % w.tiles[1], b / w.tiles[1], w.part[1], w.bpart[1]);
    return;
  }
  b -= w.tiles[1] * w.ns[1];
  wgrad_block<NOP, NH>(w.At[2], w.Bt[2], ld, w.chunk[2], b % w.tiles[2], b / w.tiles[2], w.part[2], w.bpart[2]);
}

// Sum of the splits into the parameter-shaped gradient: rows x cols of the padded product,
// keeping rows < keep_r and columns < keep_c, row-major at dst; bias sums to dst_b.  Outputs
// are numbered weights first (keep_r * keep_c), then biases (keep_r); a workgroup takes 64 of
// them, its four wavefronts sum every fourth split in double, and the four sums are added in
// a fixed order, so the result does not depend on scheduling.
struct ReduceJob {
  const float* part;
  const float* bpart;
  int ns, M, N, keep_r, keep_c;
  float* dst;
  float* dst_b;
};

// Workgroups a reduction job needs: 64 outputs each.
__host__ __device__ inline int reduce_wgs(const ReduceJob& j) { return (j.keep_r * j.keep_c + j.keep_r + 63) / 64; }

// The split sums of the three products in one launch: the workgroups of job p follow those of
// the jobs before it.
struct ReduceSet {
  ReduceJob j[3];
};

__global__ void __launch_bounds__(256) reduce_all(ReduceSet r) {
  __shared__ double red[4][64];
  int b = blockIdx.x, p = 0;
  while (p < 2 && b >= reduce_wgs(r.j[p])) b -= reduce_wgs(r.j[p++]);
  const ReduceJob& J = r.j[p];
  const float* __restrict__ part = J.part;
  const float* __restrict__ bpart = J.bpart;
  const int ns = J.ns, M = J.M, N = J.N, keep_r = J.keep_r, keep_c = J.keep_c;
  float* __restrict__ dst = J.dst;
  float* __restrict__ dst_b = J.dst_b;
  const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = b * 64 + l, nw = keep_r * keep_c;
  const float* src = nullptr;
  size_t stride = 0;
  if (i < nw) {
    src = part + (size_t)(i / keep_c) * N + i % keep_c;
    stride = (size_t)M * N;
  } else if (i < nw + keep_r) {
    src = bpart + (i - nw);
    stride = M;
  }
  double acc = 0.0;
  if (src) {
#pragma unroll 4
    for (int k = g; k < ns; k += 4) acc += src[(size_t)k * stride];
  }
  red[g][l] = acc;
  __syncthreads();
  if (g == 0 && src) {
    const double t = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
    if (i < nw) dst[i] = (float)t;
    else dst_b[i - nw] = (float)t;
  }
}

// One 32-entry bfloat16 row (64 bytes, 16-byte aligned) from packed pairs, as four 16-byte stores.
__device__ __forceinline__ void store_row(u16* row, const uint32_t (&w)[KX / 2]) {
  uint4* q = reinterpret_cast<uint4*>(row);
#pragma unroll
  for (int k = 0; k < KX / 8; ++k) q[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

// Standardised, bfloat16-rounded input rows (and their transpose) from raw float64 features;
// rows >= n are zero.
__global__ void standardise(const double* __restrict__ F, int n, int rows, const double* __restrict__ mean,
                            const double* __restrict__ sd, u16* __restrict__ X, u16* __restrict__ XT) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  uint32_t w[KX / 2];
#pragma unroll
  for (int c = 0; c < KX; ++c) {
    u16 h = 0;
    if (r < n && c < NI) h = bf16_bits((float)((F[(size_t)r * NI + c] - mean[c]) / sd[c]));
    XT[(size_t)c * rows + r] = h;
    if (c & 1) w[c / 2] |= (uint32_t)h << 16;
    else w[c / 2] = h;
  }
  store_row(X + (size_t)r * KX, w);
}

// Squared-error loss against standardised targets T/ystd and its gradient 2 (y - t)/n, rounded
// to bfloat16 into dY [rows][32] and dYT [16][rows] (zero padding); per-block loss sums.
__global__ void __launch_bounds__(256) loss_grad(const float* __restrict__ Y, const double* __restrict__ T,
                                                 const double* __restrict__ ystd, int n, int rows,
                                                 u16* __restrict__ dY, u16* __restrict__ dYT, double* __restrict__ lpart) {
  __shared__ double red[256];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  double ls = 0.0;
  if (r < rows) {
    uint32_t w[KX / 2];
#pragma unroll
    for (int c = 0; c < KX; ++c) {
      u16 h = 0;
      if (r < n && c < NO) {
        const double t = (double)(float)(T[(size_t)r * NO + c] / ystd[c]);
        const double d = (double)Y[(size_t)r * NO + c] - t;
        ls += d * d;
        h = bf16_bits((float)(2.0 * d / n));
      }
      if (c < NOP) dYT[(size_t)c * rows + r] = h;
      if (c & 1) w[c / 2] |= (uint32_t)h << 16;
      else w[c / 2] = h;
    }
    store_row(dY + (size_t)r * KX, w);
  }
  red[threadIdx.x] = ls;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// Rows of a mini-batch: Fb[r] = F[perm[b0 + r]], Tb[r] = T[perm[b0 + r]], r < nb.  An index
// outside 0..n-1 raises *bad and reads row 0 instead.
__global__ void gather_batch(const double* __restrict__ F, const double* __restrict__ T, const int* __restrict__ perm,
                             int n, int b0, int nb, double* __restrict__ Fb, double* __restrict__ Tb,
                             int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * (NI + NO)) return;
  const int r = i / (NI + NO), c = i % (NI + NO);
  int p = perm[b0 + r];
  if (p < 0 || p >= n) {
    *bad = 1;
    p = 0;
  }
  if (c < NI) Fb[(size_t)r * NI + c] = F[(size_t)p * NI + c];
  else Tb[(size_t)r * NO + (c - NI)] = T[(size_t)p * NO + (c - NI)];
}

// bfloat16 operand copies of the master weights, as prepare_weights writes them.
struct WeightCopies {
  u16 *W1b, *W2b, *W2tb, *W3b, *W3tb;
};

// Adam on the float32 master weights (bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t),
// writing each updated weight's bfloat16 copies (the zero padding of the copies is left as
// prepare_weights wrote it).  If lacc is given, thread 0 also adds the batch loss, the block
// sums lpart[0..nblk) in block order over nrows, to *lacc.
__global__ void adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                     int n, float lr, float b1, float b2, float eps, float c1, float c2, WeightCopies wc,
                     const double* __restrict__ lpart, int nblk, int nrows, double* __restrict__ lacc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (lacc && i == 0) {
    double L = 0.0;
    for (int k = 0; k < nblk; ++k) L += lpart[k];
    lacc[0] += L / nrows;
  }
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pn = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pn;
  const u16 h = bf16_bits(pn);
  if (i < OFF_B1) {
    wc.W1b[(i / NI) * KX + i % NI] = h;
  } else if (i >= OFF_W2 && i < OFF_B2) {
    const int k = i - OFF_W2;
    wc.W2b[k] = h;
    wc.W2tb[(k % NH) * NH + k / NH] = h;
  } else if (i >= OFF_W3 && i < OFF_B3) {
    const int k = i - OFF_W3;
    wc.W3b[k] = h;
    wc.W3tb[(k % NH) * KX + k / NH] = h;
  }
}

// bfloat16 operand copies of the master weights: W1 [256][32], W2 [256][256], W2^T, W3 [16][256],
// W3^T [256][32] (zero padding).
__global__ void prepare_weights(const float* __restrict__ P, u16* __restrict__ W1b, u16* __restrict__ W2b,
                                u16* __restrict__ W2tb, u16* __restrict__ W3b, u16* __restrict__ W3tb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NH * NH) {
    const int r = i / NH, c = i % NH;
    W2b[i] = bf16_bits(P[OFF_W2 + i]);
    W2tb[(size_t)c * NH + r] = bf16_bits(P[OFF_W2 + i]);
  }
  if (i < NH * KX) {
    const int r = i / KX, c = i % KX;
    W1b[i] = c < NI ? bf16_bits(P[OFF_W1 + r * NI + c]) : 0;
    W3tb[i] = c < NO ? bf16_bits(P[OFF_W3 + c * NH + r]) : 0;
  }
  if (i < NOP * NH) {
    const int r = i / NH, c = i % NH;
    W3b[i] = r < NO ? bf16_bits(P[OFF_W3 + r * NH + c]) : 0;
  }
}

// Sums and sums of squares of the 29 feature and target columns over a data set, in two
// passes: each of MOM_BLOCKS workgroups reads whole rows in a grid-stride loop (so the rows
// are read once, in order) and writes its partial sums part[b][c][0..1]; then one workgroup
// adds the partials.
constexpr int MOM_BLOCKS = 1024, NC = NI + NO;

__global__ void __launch_bounds__(256) column_moments(const double* __restrict__ F, const double* __restrict__ T,
                                                      int n, double* __restrict__ part) {
  __shared__ double red[4][NC][2];
  double a[NC], q[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) a[c] = q[c] = 0.0;
  for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < (size_t)n; r += (size_t)gridDim.x * blockDim.x) {
    const double2* f = reinterpret_cast<const double2*>(F + r * NI);   // rows of 208 bytes
#pragma unroll
    for (int c = 0; c < NI / 2; ++c) {
      const double2 x = f[c];
      a[2 * c] += x.x;
      q[2 * c] += x.x * x.x;
      a[2 * c + 1] += x.y;
      q[2 * c + 1] += x.y * x.y;
    }
#pragma unroll
    for (int c = 0; c < NO; ++c) {
      const double x = T[r * NO + c];
      a[NI + c] += x;
      q[NI + c] += x * x;
    }
  }
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double x = a[c], y = q[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      x += __shfl_xor(x, o, 64);
      y += __shfl_xor(y, o, 64);
    }
    if (l == 0) {
      red[w][c][0] = x;
      red[w][c][1] = y;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * NC) {
    const int c = threadIdx.x >> 1, k = threadIdx.x & 1;
    part[((size_t)blockIdx.x * NC + c) * 2 + k] = (red[0][c][k] + red[1][c][k]) + (red[2][c][k] + red[3][c][k]);
  }
}

// Total of the partials: eight wavefronts each add every eighth block's partials, and the
// eight sums are added in a fixed order.
__global__ void __launch_bounds__(512) moments_total(const double* __restrict__ part, int nblk,
                                                     double* __restrict__ out /*[29][2]*/) {
  __shared__ double red[8][2 * NC];
  const int i = threadIdx.x & 63, g = threadIdx.x >> 6;
  double s = 0.0;
  if (i < 2 * NC) {
#pragma unroll 8
    for (int b = g; b < nblk; b += 8) s += part[(size_t)b * 2 * NC + i];
    red[g][i] = s;
  }
  __syncthreads();
  if (g == 0 && i < 2 * NC)
    out[i] = ((red[0][i] + red[1][i]) + (red[2][i] + red[3][i])) + ((red[4][i] + red[5][i]) + (red[6][i] + red[7][i]));
}

// ---------------------------------------------------------------------------
// features and prediction on a simulation's state (one row per chain node)
// ---------------------------------------------------------------------------

// Raw features of chain node entry i (missing neighbours of a rod end replicated):
// v_{i-1} - v_i, v_{i+1} - v_i, v_i, a_i = v_i - v_prev_i (velocity change over the last
// step), x_{i-1} - 2 x_i + x_{i+1}, log10 E, radius, mean rest length of the edges at i, the
// natural curvature at i in 1/m (nearest interior node at the ends), j_i = a_i - (v_prev_i -
// v_prev2_i) (the change of the velocity change) and a_{i-1} - 2 a_i + a_{i+1}.
__global__ void node_features(DmDev D, int rows, const int* __restrict__ cn_chain, const double* __restrict__ nconst,
                              double* __restrict__ F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const int NN = D.n_nodes_tot, NS = D.n_st_tot;
  const int c = cn_chain[i];
  const DmChain ch = D.chain[c];
  const int k = i - ch.node_tab, N = ch.n_nodes;
  const int n0 = D.chain_node[ch.node_tab + k];
  const int nm = D.chain_node[ch.node_tab + (k >= 1 ? k - 1 : k)];
  const int np = D.chain_node[ch.node_tab + (k <= N - 2 ? k + 1 : k)];
  double* f = F + (size_t)i * NI;
  for (int q = 0; q < 3; ++q) {
    const double vi = D.v[q * NN + n0], ai = vi - D.vprev[q * NN + n0];
    f[q] = D.v[q * NN + nm] - vi;
    f[3 + q] = D.v[q * NN + np] - vi;
    f[6 + q] = vi;
    f[9 + q] = ai;
    f[12 + q] = D.x0[q * NN + nm] - 2.0 * D.x0[q * NN + n0] + D.x0[q * NN + np];
    f[20 + q] = ai - (D.vprev[q * NN + n0] - D.vprev2[q * NN + n0]);
    f[23 + q] = (D.v[q * NN + nm] - D.vprev[q * NN + nm]) - 2.0 * ai + (D.v[q * NN + np] - D.vprev[q * NN + np]);
  }
  for (int q = 0; q < 3; ++q) f[15 + q] = nconst[(size_t)i * 3 + q];
  if (N >= 3) {
    const int kc = k < 1 ? 1 : (k > N - 2 ? N - 2 : k);
    const int s = ch.st_off + kc - 1;
    f[18] = D.kbar[s] / D.Vbar[s];
    f[19] = D.kbar[NS + s] / D.Vbar[s];
  } else {
    f[18] = f[19] = 0.0;
  }
}

// Training targets after a step: the displacement beyond the third-order extrapolation,
// dt (v_{n+1} - v_n - a_n - j_n), with v_n, a_n and j_n read from the step-start features.
__global__ void node_targets(DmDev D, int rows, const double* __restrict__ Fprev, double dt, double* __restrict__ T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const int NN = D.n_nodes_tot;
  const int n0 = D.chain_node[i];
  for (int q = 0; q < 3; ++q) {
    const double* f = Fprev + (size_t)i * NI;
    T[(size_t)i * NO + q] = dt * (D.v[q * NN + n0] - f[6 + q] - f[9 + q] - f[20 + q]);   // f: v_n, a_n, j_n
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {
thread_local std::string g_mlp_err;
dm_status mfail(dm_status s, const std::string& m) { g_mlp_err = m; return s; }
#define MH(call)                                                                                  \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) return mfail(DM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
int rup(int a, int b) { return (a + b - 1) / b * b; }
}  // namespace

struct dm_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  int max_rows = 0;                       // padded row capacity (multiple of 64)
  std::vector<void*> allocs;
  float *P = nullptr, *M = nullptr, *V = nullptr, *G = nullptr, *Y = nullptr, *part = nullptr, *bpart = nullptr;
  u16 *W1b = nullptr, *W2b = nullptr, *W2tb = nullptr, *W3b = nullptr, *W3tb = nullptr;
  u16 *X = nullptr, *XT = nullptr, *H1 = nullptr, *H1T = nullptr, *H2 = nullptr, *H2T = nullptr;
  u16 *dY = nullptr, *dYT = nullptr, *dH2 = nullptr, *dH2T = nullptr, *dH1T = nullptr;
  double *mean = nullptr, *sd = nullptr, *ystd = nullptr, *lpart = nullptr, *moments = nullptr;
  double *Fb = nullptr, *Tb = nullptr, *lacc = nullptr;   // gathered mini-batch, epoch loss sum
  int* bad = nullptr;                                      // raised by an out-of-range batch index
  double* mpart = nullptr;                                 // per-workgroup column moments
  int t = 0;
};

namespace {

template <class T>
dm_status malloc_n(dm_mlp* m, T** p, size_t n) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return mfail(DM_ERR_OOM, "dm_mlp: hipMalloc failed");
  m->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return hipMemset(q, 0, std::max<size_t>(n, 1) * sizeof(T)) == hipSuccess ? DM_OK : mfail(DM_ERR_HIP, "hipMemset");
}

dm_status check_rows(const dm_mlp* m, int n) {
  if (!m) return mfail(DM_ERR_INVALID_ARG, "null network");
  if (n <= 0 || n > m->max_rows) return mfail(DM_ERR_INVALID_ARG, "dm_mlp: row count outside 1..max_rows");
  return DM_OK;
}

// Activations of a forward pass: standardised inputs, both hidden layers (row-major and
// transposed), outputs.
struct FwdBufs {
  u16 *X, *XT, *H1, *H1T, *H2, *H2T;
  float* Y;
};

// Forward pass on raw features F (device, [n][26]) into the activation buffers b (rows padded
// to ROWS_PAD): leaves Y [rows][3] (standardised outputs) and every activation needed by the
// backward pass.
dm_status forward_into(dm_mlp* m, const FwdBufs& b, const double* F, int n, int rows) {
  hipStream_t st = m->stream;
  hipLaunchKernelGGL(standardise, dim3((rows + 255) / 256), dim3(256), 0, st, F, n, rows, m->mean, m->sd, b.X, b.XT);
  const dim3 blk(256);
  hipLaunchKernelGGL((row_gemm<KX, NH, EPI_HIDDEN>), dim3(row_grid<KX, NH>(rows)), blk, 0, st, b.X, m->W1b,
                     m->P + OFF_B1, nullptr, rows, b.H1, b.H1T, nullptr);
  hipLaunchKernelGGL((row_gemm<NH, NH, EPI_HIDDEN>), dim3(row_grid<NH, NH>(rows)), blk, 0, st, b.H1, m->W2b,
                     m->P + OFF_B2, nullptr, rows, b.H2, b.H2T, nullptr);
  hipLaunchKernelGGL((row_gemm<NH, NOP, EPI_OUTPUT>), dim3(row_grid<NH, NOP>(rows)), blk, 0, st, b.H2, m->W3b,
                     m->P + OFF_B3, nullptr, rows, nullptr, nullptr, b.Y);
  MH(hipGetLastError());
  return DM_OK;
}

// The same into the network's own buffers.
dm_status forward_rows(dm_mlp* m, const double* F, int n, int rows) {
  return forward_into(m, FwdBufs{m->X, m->XT, m->H1, m->H1T, m->H2, m->H2T, m->Y}, F, n, rows);
}

// ---- activations of dm_mlp_forward_noalloc: a file-scope device array, one copy per GPU ----
// Byte offsets of the buffers for DM_MLP_NOALLOC_MAX_ROWS rows (each a multiple of 256).
constexpr size_t NA_ROWS = DM_MLP_NOALLOC_MAX_ROWS;
constexpr size_t NA_X = 0, NA_XT = NA_X + NA_ROWS * KX * 2, NA_H1 = NA_XT + NA_ROWS * KX * 2;
constexpr size_t NA_H1T = NA_H1 + NA_ROWS * NH * 2, NA_H2 = NA_H1T + NA_ROWS * NH * 2;
constexpr size_t NA_H2T = NA_H2 + NA_ROWS * NH * 2, NA_Y = NA_H2T + NA_ROWS * NH * 2;
constexpr size_t NA_BYTES = NA_Y + NA_ROWS * NO * 4;
static_assert(NA_ROWS % ROWS_PAD == 0 && NA_Y % 256 == 0, "scratch layout");
}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {
// Device address of `scratch` on each device, taken once per device (with that device
// current) by hipGetSymbolAddress; host code uses only these addresses.
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

dm_status scratch_address(int device, void** out) {
  if (device < 0 || device >= 64) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_forward_noalloc: device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return mfail(DM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return DM_OK;
}

dm_status prepare(dm_mlp* m) {
  hipLaunchKernelGGL(prepare_weights, dim3((NH * NH + 255) / 256), dim3(256), 0, m->stream, m->P, m->W1b, m->W2b,
                     m->W2tb, m->W3b, m->W3tb);
  MH(hipGetLastError());
  return DM_OK;
}

// Adam step on m->G (bias corrections from the step count) with the bfloat16 weight copies;
// with lacc, the batch loss of the last gradient pass (nrows rows) is added to *lacc.
dm_status adam_step(dm_mlp* m, float lr, int nrows = 0, double* lacc = nullptr) {
  m->t += 1;
  const float c1 = (float)(1.0 - std::pow(0.9, m->t)), c2 = (float)(1.0 - std::pow(0.999, m->t));
  const WeightCopies wc{m->W1b, m->W2b, m->W2tb, m->W3b, m->W3tb};
  const int nblk = (rup(std::max(nrows, 1), ROWS_PAD) + 255) / 256;
  hipLaunchKernelGGL(adam, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->P, m->M, m->V, m->G, NPARAM, lr,
                     0.9f, 0.999f, 1e-8f, c1, c2, wc, m->lpart, nblk, nrows, lacc);
  MH(hipGetLastError());
  return DM_OK;
}

// Loss and gradients into m->G for rows 0..n-1 of raw features F and raw targets T.
dm_status gradients(dm_mlp* m, const double* F, const double* T, int n, double* loss) {
  const int rows = rup(n, ROWS_PAD);
  dm_status s;
  if ((s = forward_rows(m, F, n, rows)) != DM_OK) return s;
  hipStream_t st = m->stream;
  const int nb = (rows + 255) / 256;
  hipLaunchKernelGGL(loss_grad, dim3(nb), dim3(256), 0, st, m->Y, T, m->ystd, n, rows, m->dY, m->dYT, m->lpart);
  const dim3 b(256);
  hipLaunchKernelGGL((row_gemm<KX, NH, EPI_DGRAD>), dim3(row_grid<KX, NH>(rows)), b, 0, st, m->dY, m->W3tb, nullptr,
                     m->H2, rows, m->dH2, m->dH2T, nullptr);
  hipLaunchKernelGGL((row_gemm<NH, NH, EPI_DGRAD>), dim3(row_grid<NH, NH>(rows)), b, 0, st, m->dH2, m->W2tb, nullptr,
                     m->H1, rows, nullptr, m->dH1T, nullptr);
  float* G = m->G;
  // The three weight-gradient products (W2, W1, W3; tiles = (M / 16) x (N / min(N, 64))), each
  // with its own split plan and partial-sum region, then their split sums.
  WgradSet w;
  ReduceSet r;
  const u16* At[3] = {m->dH2T, m->dH1T, m->dYT};
  const u16* Bt[3] = {m->H1T, m->XT, m->H2T};
  const int Ms[3] = {NH, NH, NOP}, Ns[3] = {NH, KX, NH}, tiles[3] = {(NH / 16) * (NH / 64), NH / 16, NH / 64};
  const int kr[3] = {NH, NH, NO}, kc[3] = {NH, NI, NH};
  float* dst[3] = {G + OFF_W2, G + OFF_W1, G + OFF_W3};
  float* dstb[3] = {G + OFF_B2, G + OFF_B1, G + OFF_B3};
  float* part = m->part;
  float* bpart = m->bpart;
  int wblocks = 0, rblocks = 0;
  for (int q = 0; q < 3; ++q) {
    w.At[q] = At[q];
    w.Bt[q] = Bt[q];
    w.part[q] = part;
    w.bpart[q] = bpart;
    w.tiles[q] = tiles[q];
    split_plan(rows, tiles[q], &w.chunk[q], &w.ns[q]);
    r.j[q] = ReduceJob{part, bpart, w.ns[q], Ms[q], Ns[q], kr[q], kc[q], dst[q], dstb[q]};
    part += (size_t)NS_MAX * Ms[q] * Ns[q];
    bpart += (size_t)NS_MAX * Ms[q];
    wblocks += tiles[q] * w.ns[q];
    rblocks += reduce_wgs(r.j[q]);
  }
  hipLaunchKernelGGL(wgrad_all, dim3(wblocks), dim3(64), 0, st, w, rows);
  hipLaunchKernelGGL(reduce_all, dim3(rblocks), dim3(256), 0, st, r);
  MH(hipGetLastError());
  if (loss) {
    std::vector<double> lp(nb);
    MH(hipMemcpyAsync(lp.data(), m->lpart, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    MH(hipStreamSynchronize(st));
    double L = 0.0;
    for (double v : lp) L += v;
    *loss = L / n;
  }
  return DM_OK;
}

}  // namespace

extern "C" {

size_t dm_mlp_num_params(void) { return NPARAM; }
int dm_mlp_num_inputs(void) { return NI; }
const char* dm_mlp_last_error(void) { return g_mlp_err.c_str(); }

dm_status dm_mlp_create(int device, void* stream, int max_rows, dm_mlp** out) {
  if (!out || max_rows <= 0) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_create: bad arguments");
  MH(hipSetDevice(device));
  dm_mlp* m = new dm_mlp();
  m->device = device;
  m->stream = (hipStream_t)stream;
  m->max_rows = rup(max_rows, ROWS_PAD);
  const size_t R = m->max_rows;
  dm_status s = DM_OK;
  auto A = [&](auto** p, size_t n) { if (s == DM_OK) s = malloc_n(m, p, n); };
  A(&m->P, NPARAM); A(&m->M, NPARAM); A(&m->V, NPARAM); A(&m->G, NPARAM); A(&m->Y, R * NO);
  A(&m->part, (size_t)NS_MAX * (NH * NH + NH * KX + NOP * NH)); A(&m->bpart, (size_t)NS_MAX * (2 * NH + NOP));
  A(&m->W1b, NH * KX); A(&m->W2b, NH * NH); A(&m->W2tb, NH * NH); A(&m->W3b, NOP * NH); A(&m->W3tb, NH * KX);
  A(&m->X, R * KX); A(&m->XT, R * KX); A(&m->H1, R * NH); A(&m->H1T, R * NH); A(&m->H2, R * NH); A(&m->H2T, R * NH);
  A(&m->dY, R * KX); A(&m->dYT, R * NOP); A(&m->dH2, R * NH); A(&m->dH2T, R * NH); A(&m->dH1T, R * NH);
  A(&m->mean, NI); A(&m->sd, NI); A(&m->ystd, NO); A(&m->lpart, R / 256 + 1); A(&m->moments, 2 * (NI + NO));
  A(&m->Fb, R * NI); A(&m->Tb, R * NO); A(&m->lacc, 1); A(&m->bad, 1);
  A(&m->mpart, (size_t)MOM_BLOCKS * 2 * (NI + NO));
  if (s != DM_OK) { dm_mlp_destroy(m); return s; }
  std::vector<double> one(NI, 1.0);
  if (hipMemcpy(m->sd, one.data(), sizeof(double) * NI, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->ystd, one.data(), sizeof(double) * NO, hipMemcpyHostToDevice) != hipSuccess) {
    dm_mlp_destroy(m);
    return mfail(DM_ERR_HIP, "dm_mlp_create: hipMemcpy");
  }
  *out = m;
  return DM_OK;
}

dm_status dm_mlp_set_params(dm_mlp* m, const float* params, int on_device) {
  if (!m || !params) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_set_params: null argument");
  MH(hipSetDevice(m->device));
  MH(hipMemcpyAsync(m->P, params, sizeof(float) * NPARAM, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                    m->stream));
  MH(hipMemsetAsync(m->M, 0, sizeof(float) * NPARAM, m->stream));
  MH(hipMemsetAsync(m->V, 0, sizeof(float) * NPARAM, m->stream));
  m->t = 0;
  dm_status s = prepare(m);
  MH(hipStreamSynchronize(m->stream));
  return s;
}

dm_status dm_mlp_get_params(dm_mlp* m, float* params, int on_device) {
  if (!m || !params) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_get_params: null argument");
  MH(hipMemcpyAsync(params, m->P, sizeof(float) * NPARAM, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                    m->stream));
  MH(hipStreamSynchronize(m->stream));
  return DM_OK;
}

dm_status dm_mlp_set_normalisation(dm_mlp* m, const double* mean, const double* sd, const double* ystd) {
  if (!m || !mean || !sd || !ystd) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_set_normalisation: null argument");
  for (int i = 0; i < NI; ++i)
    if (!(sd[i] > 0) || !std::isfinite(mean[i])) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_set_normalisation: bad value");
  for (int i = 0; i < NO; ++i)
    if (!(ystd[i] > 0)) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_set_normalisation: bad value");
  MH(hipMemcpy(m->mean, mean, sizeof(double) * NI, hipMemcpyHostToDevice));
  MH(hipMemcpy(m->sd, sd, sizeof(double) * NI, hipMemcpyHostToDevice));
  MH(hipMemcpy(m->ystd, ystd, sizeof(double) * NO, hipMemcpyHostToDevice));
  return DM_OK;
}

dm_status dm_mlp_get_normalisation(dm_mlp* m, double* mean, double* sd, double* ystd) {
  if (!m || !mean || !sd || !ystd) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_get_normalisation: null argument");
  MH(hipMemcpy(mean, m->mean, sizeof(double) * NI, hipMemcpyDeviceToHost));
  MH(hipMemcpy(sd, m->sd, sizeof(double) * NI, hipMemcpyDeviceToHost));
  MH(hipMemcpy(ystd, m->ystd, sizeof(double) * NO, hipMemcpyDeviceToHost));
  return DM_OK;
}

dm_status dm_mlp_fit_normalisation(dm_mlp* m, const double* F, const double* T, int n) {
  if (!m || !F || !T || n < 2) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_fit_normalisation: bad arguments");
  if (reinterpret_cast<uintptr_t>(F) % 16 != 0)
    return mfail(DM_ERR_INVALID_ARG, "dm_mlp_fit_normalisation: F is not 16-byte aligned");
  MH(hipSetDevice(m->device));
  hipLaunchKernelGGL(column_moments, dim3(MOM_BLOCKS), dim3(256), 0, m->stream, F, T, n, m->mpart);
  hipLaunchKernelGGL(moments_total, dim3(1), dim3(512), 0, m->stream, m->mpart, MOM_BLOCKS, m->moments);
  MH(hipGetLastError());
  std::vector<double> mo(2 * (NI + NO));
  MH(hipMemcpyAsync(mo.data(), m->moments, sizeof(double) * mo.size(), hipMemcpyDeviceToHost, m->stream));
  MH(hipStreamSynchronize(m->stream));
  double mean[NI], sd[NI], ys[NO];
  for (int c = 0; c < NI + NO; ++c) {
    const double mu = mo[2 * c] / n;
    const double var = std::max(mo[2 * c + 1] / n - mu * mu, 0.0);
    const double s = var > 1e-30 * std::max(1.0, mu * mu) ? std::sqrt(var) : 1.0;
    if (c < NI) { mean[c] = mu; sd[c] = s; }
    else ys[c - NI] = std::sqrt(mo[2 * c + 1] / n) > 0 ? std::sqrt(mo[2 * c + 1] / n) : 1.0;
  }
  return dm_mlp_set_normalisation(m, mean, sd, ys);
}

dm_status dm_mlp_forward_noalloc(dm_mlp* m, const double* F, int n, float* Y) {
  if (!m || !F || !Y) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_forward_noalloc: null argument");
  if (n <= 0 || n > DM_MLP_NOALLOC_MAX_ROWS)
    return mfail(DM_ERR_INVALID_ARG, "dm_mlp_forward_noalloc: row count outside 1.." +
                                         std::to_string(DM_MLP_NOALLOC_MAX_ROWS) + " (the static activation buffer)");
  MH(hipSetDevice(m->device));
  void* base = nullptr;
  dm_status s;
  if ((s = scratch_address(m->device, &base)) != DM_OK) return s;
  unsigned char* p = static_cast<unsigned char*>(base);
  const FwdBufs b{reinterpret_cast<u16*>(p + NA_X), reinterpret_cast<u16*>(p + NA_XT),
                  reinterpret_cast<u16*>(p + NA_H1), reinterpret_cast<u16*>(p + NA_H1T),
                  reinterpret_cast<u16*>(p + NA_H2), reinterpret_cast<u16*>(p + NA_H2T),
                  reinterpret_cast<float*>(p + NA_Y)};
  if ((s = forward_into(m, b, F, n, rup(n, ROWS_PAD))) != DM_OK) return s;
  MH(hipMemcpyAsync(Y, b.Y, sizeof(float) * NO * (size_t)n, hipMemcpyDeviceToDevice, m->stream));
  MH(hipStreamSynchronize(m->stream));
  return DM_OK;
}

dm_status dm_mlp_forward(dm_mlp* m, const double* F, int n, float* Y) {
  dm_status s;
  if ((s = check_rows(m, n)) != DM_OK) return s;
  if (!F || !Y) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_forward: null argument");
  MH(hipSetDevice(m->device));
  if ((s = forward_rows(m, F, n, rup(n, ROWS_PAD))) != DM_OK) return s;
  MH(hipMemcpyAsync(Y, m->Y, sizeof(float) * NO * (size_t)n, hipMemcpyDeviceToDevice, m->stream));
  MH(hipStreamSynchronize(m->stream));
  return DM_OK;
}

dm_status dm_mlp_gradients(dm_mlp* m, const double* F, const double* T, int n, float* grads, double* loss) {
  dm_status s;
  if ((s = check_rows(m, n)) != DM_OK) return s;
  if (!F || !T || !grads) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_gradients: null argument");
  MH(hipSetDevice(m->device));
  if ((s = gradients(m, F, T, n, loss)) != DM_OK) return s;
  MH(hipMemcpyAsync(grads, m->G, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, m->stream));
  MH(hipStreamSynchronize(m->stream));
  return DM_OK;
}

dm_status dm_mlp_train_step(dm_mlp* m, const double* F, const double* T, int n, float lr, double* loss) {
  dm_status s;
  if ((s = check_rows(m, n)) != DM_OK) return s;
  if (!F || !T || !(lr > 0)) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_train_step: bad arguments");
  MH(hipSetDevice(m->device));
  if ((s = gradients(m, F, T, n, loss)) != DM_OK) return s;
  return adam_step(m, lr);
}

dm_status dm_mlp_train_epoch(dm_mlp* m, const double* F, const double* T, const int* perm, int n, int batch,
                             float lr, double* mean_loss) {
  dm_status s;
  if ((s = check_rows(m, batch)) != DM_OK) return s;
  if (!F || !T || !perm || batch > n || !(lr > 0)) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_train_epoch: bad arguments");
  MH(hipSetDevice(m->device));
  hipStream_t st = m->stream;
  MH(hipMemsetAsync(m->lacc, 0, sizeof(double), st));
  MH(hipMemsetAsync(m->bad, 0, sizeof(int), st));
  const int nbatch = n / batch;
  const int items = batch * (NI + NO);
  for (int k = 0; k < nbatch; ++k) {
    hipLaunchKernelGGL(gather_batch, dim3((items + 255) / 256), dim3(256), 0, st, F, T, perm, n, k * batch, batch,
                       m->Fb, m->Tb, m->bad);
    if ((s = gradients(m, m->Fb, m->Tb, batch, nullptr)) != DM_OK) return s;
    if ((s = adam_step(m, lr, batch, m->lacc)) != DM_OK) return s;
  }
  double L = 0.0;
  int bad = 0;
  MH(hipMemcpyAsync(&L, m->lacc, sizeof(double), hipMemcpyDeviceToHost, st));
  MH(hipMemcpyAsync(&bad, m->bad, sizeof(int), hipMemcpyDeviceToHost, st));
  MH(hipStreamSynchronize(st));
  if (bad) return mfail(DM_ERR_INVALID_ARG, "dm_mlp_train_epoch: perm holds an index outside 0..n-1");
  if (mean_loss) *mean_loss = L / nbatch;
  return DM_OK;
}

void dm_mlp_destroy(dm_mlp* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipStreamSynchronize(m->stream);
  for (void* p : m->allocs) (void)hipFree(p);
  delete m;
}

// --- used by the simulation runtime --------------------------------------------------------

int dm_mlp_capacity(const dm_mlp* m) { return m ? m->max_rows : 0; }

hipError_t dm_ws_launch_features(const DmDev* D, int rows, const int* cn_chain, const double* nconst, double* F,
                                 hipStream_t st) {
  hipLaunchKernelGGL(node_features, dim3((rows + 255) / 256), dim3(256), 0, st, *D, rows, cn_chain, nconst, F);
  return hipGetLastError();
}

hipError_t dm_ws_launch_targets(const DmDev* D, int rows, const int* cn_chain, const double* Fprev, double dt,
                                double* T, hipStream_t st) {
  (void)cn_chain;
  hipLaunchKernelGGL(node_targets, dim3((rows + 255) / 256), dim3(256), 0, st, *D, rows, Fprev, dt, T);
  return hipGetLastError();
}

}  // extern "C"

#ifndef __HIP_DEVICE_COMPILE__
void dm_mlp_view(const dm_mlp* m, DmNetView* v) {
  *v = DmNetView{m->W1b, m->W2b, m->W3b, m->P + OFF_B1, m->P + OFF_B2, m->P + OFF_B3, m->mean, m->sd, m->ystd};
}
#endif
