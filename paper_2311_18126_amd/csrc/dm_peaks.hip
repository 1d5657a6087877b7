// Measured ceilings of the GPU that the roofline figures are quoted against, next to the
// published ones: FP64 vector FMA throughput, device-to-device copy bandwidth through HBM and
// dense BF16 matrix-core throughput.  Standalone program (no part of libdmrod.so); prints one
// JSON line.  Every kernel writes one value per thread so that none of its work is removed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                        \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));               \
      std::exit(2);                                                                     \
    }                                                                                   \
  } while (0)

constexpr int kChains = 8;  // independent FMA chains per lane (hides the FP64 FMA latency)

// kChains x iters dependent FMAs per lane; the multiplier is just below one so values stay
// finite.  Flops per launch = 2 * kChains * iters * threads.
__global__ __launch_bounds__(256) void fma_f64(double* out, int iters, double m) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  double a[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) a[c] = 1.0 + 1e-3 * (c + (gid & 7));
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = __builtin_fma(a[c], m, 1e-7);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += a[c];
  out[gid] = s;
}

// Grid-stride copy of n 16-byte elements.
__global__ __launch_bounds__(256) void copy16(const double2* __restrict__ src,
                                              double2* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kAcc = 4;  // independent accumulators per wavefront

// kAcc x iters dependent 16x16x32 BF16 products per wavefront (16384 flops each), operands
// held in registers.
__global__ __launch_bounds__(256) void mfma_bf16(float* out, int iters) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  bf16x8 a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(1e-3f * (float)((threadIdx.x + j) & 15));
    b[j] = (__bf16)(1e-3f * (float)((threadIdx.x * 3 + j) & 15));
  }
  f32x4 acc[kAcc];
#pragma unroll
  for (int c = 0; c < kAcc; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kAcc; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kAcc; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[gid] = s;
}

// Best of reps timed launches (ms), after one untimed launch.
template <class F>
static float best_ms(F launch, int reps) {
  hipEvent_t t0, t1;
  CHECK(hipEventCreate(&t0));
  CHECK(hipEventCreate(&t1));
  launch();
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  float best = 1e30f;
  for (int r = 0; r < reps; ++r) {
    CHECK(hipEventRecord(t0, 0));
    launch();
    CHECK(hipEventRecord(t1, 0));
    CHECK(hipEventSynchronize(t1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, t0, t1));
    best = std::min(best, ms);
  }
  CHECK(hipEventDestroy(t0));
  CHECK(hipEventDestroy(t1));
  return best;
}

int main(int argc, char** argv) {
  const size_t copy_bytes = (argc > 1) ? std::strtoull(argv[1], nullptr, 10) : (size_t(2) << 30);
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int cus = prop.multiProcessorCount;

  // 8 workgroups of 256 lanes per CU: 8 wavefronts per SIMD.
  const int blocks = cus * 8, threads = 256;
  const size_t lanes = (size_t)blocks * threads;
  double* fout = nullptr;
  float* mout = nullptr;
  CHECK(hipMalloc(&fout, lanes * sizeof(double)));
  CHECK(hipMalloc(&mout, lanes * sizeof(float)));

  const int fma_iters = 1 << 14;
  const float fma_ms = best_ms([&] { fma_f64<<<blocks, threads>>>(fout, fma_iters, 0.9999999); }, 5);
  const double fma_tflops = 2.0 * kChains * fma_iters * (double)lanes / (fma_ms * 1e-3) / 1e12;

  const int mfma_iters = 1 << 14;
  const float mfma_ms = best_ms([&] { mfma_bf16<<<blocks, threads>>>(mout, mfma_iters); }, 5);
  const double waves = (double)lanes / 64.0;
  const double mfma_tflops = 16384.0 * kAcc * mfma_iters * waves / (mfma_ms * 1e-3) / 1e12;

  const size_t n16 = copy_bytes / 16;
  double2 *src = nullptr, *dst = nullptr;
  CHECK(hipMalloc(&src, n16 * 16));
  CHECK(hipMalloc(&dst, n16 * 16));
  CHECK(hipMemset(src, 0, n16 * 16));
  const int copy_blocks = cus * 16;
  const float copy_ms = best_ms([&] { copy16<<<copy_blocks, threads>>>(src, dst, n16); }, 10);
  const double copy_gbs = 2.0 * (double)(n16 * 16) / (copy_ms * 1e-3) / 1e9;

  std::printf("{\"device\": \"%s\", \"compute_units\": %d, \"clock_mhz\": %d, "
              "\"fp64_fma_tflops\": %.2f, \"fp64_fma_ms\": %.3f, "
              "\"hbm_copy_gbs\": %.1f, \"copy_bytes_each_way\": %zu, \"copy_ms\": %.3f, "
              "\"bf16_mfma_tflops\": %.1f, \"bf16_mfma_ms\": %.3f}\n",
              prop.gcnArchName, cus, prop.clockRate / 1000, fma_tflops, fma_ms, copy_gbs,
              n16 * 16, copy_ms, mfma_tflops, mfma_ms);
  CHECK(hipFree(src));
  CHECK(hipFree(dst));
  CHECK(hipFree(fout));
  CHECK(hipFree(mout));
  return 0;
}
