// Matrix-core ceiling of this GPU for the slice product's instruction mix: the figure the slice
// GEMM's achieved INT8 rate is compared with, beside the published dense peak. Every CU runs
// one block of 4 waves; each wave issues the product kernel's 128 x 128 wave tile per K-stage
// (4 x 4 accumulator blocks, two 32-deep halves: 32 v_mfma_i32_32x32x32_i8) on operands that
// change every stage, so the matrix cores see random-looking data as in the product, with
//   variant 0: operands kept in registers (flipped by a stage-dependent mask),
//   variant 1: operands read from LDS as the product reads them (16 x 16 bytes per lane and
//              stage, conflict-free), double-buffered one stage ahead,
//   variant 2: variant 1 plus the LDS writes of the product's operand ring (8 x 16 bytes per
//              lane and stage, into the stage two ahead) and a block barrier per stage.
// The product kernel itself adds the global-to-LDS operand stream on top of variant 2.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/refeig.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kStageBytes = 32768;   // one K-stage of both operands of a 256 x 256 tile
constexpr int kStages = 4;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {   // Wang-style integer hash
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

template <int VAR>
__global__ __launch_bounds__(256, 1) void k_mfma_probe(int rounds, uint32_t seed,
                                                       int32_t *__restrict__ out,
                                                       unsigned long long *__restrict__ clk) {
  __shared__ __attribute__((aligned(1024))) int8_t ring[kStages * kStageBytes];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t base = seed ^ (blockIdx.x * 256u + tid) * 0x9e3779b9u;
  if constexpr (VAR > 0) {
    // fill the ring with hashed bytes (every thread 512 bytes)
    uint32_t *w = (uint32_t *)ring;
    for (int i = tid; i < kStages * kStageBytes / 4; i += 256) w[i] = mix32(base + i);
    __syncthreads();
  }
  v4i fa[2][2][4], fb[2][2][4];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        fa[0][ks][x][e] = (int)mix32(base + 97u * (ks * 16 + x * 4 + e));
        fb[0][ks][x][e] = (int)mix32(base + 131u * (ks * 16 + x * 4 + e) + 7u);
      }
  // fragment r of a stage: wave w's 16 reads cover 16 KB, lane-contiguous 16-byte pieces
  auto frag_off = [&](int st, int which, int ks, int x) {
    return st * kStageBytes + which * 16384 + ((ks * 4 + x) * 4 + wave) * 1024 % 16384 +
           lane * 16;
  };
  auto load = [&](int r, v4i (&a)[2][4], v4i (&b)[2][4]) {
    const int st = r & (kStages - 1);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        a[ks][x] = *(const v4i *)(ring + frag_off(st, 0, ks, x));
        b[ks][x] = *(const v4i *)(ring + frag_off(st, 1, ks, x));
      }
  };
  auto flip = [&](int r, const v4i (&ca)[2][4], const v4i (&cb)[2][4], v4i (&na)[2][4],
                  v4i (&nb)[2][4]) {
    const int m = (int)(0x9e3779b9u * (uint32_t)(r + 1));
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        na[ks][x] = ca[ks][x] ^ m;
        nb[ks][x] = cb[ks][x] ^ (m >> 3);
      }
  };
  v16i acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][c][v] = 0;
  if constexpr (VAR > 0) load(0, fa[0], fb[0]);
  const unsigned long long t0 = clock64(), w0 = wall_clock64();
  auto stage = [&](int r, const v4i (&ca)[2][4], const v4i (&cb)[2][4], v4i (&na)[2][4],
                   v4i (&nb)[2][4]) {
    if constexpr (VAR == 2) {
      __syncthreads();
      // the operand ring's refill of the stage two ahead: 8 x 16 bytes per lane
      const int st = (r + 2) & (kStages - 1);
      const v4i val = ca[0][0] ^ (int)r;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        *(v4i *)(ring + st * kStageBytes + (wave * 8 + i) * 1024 + lane * 16) = val;
    }
    if constexpr (VAR > 0) load(r + 1, na, nb);
    else flip(r, ca, cb, na, nb);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ca[ks][x], cb[ks][y], acc[x][y], 0,
                                                            0, 0);
  };
  for (int r = 0; r < rounds; r += 2) {
    stage(r, fa[0], fb[0], fa[1], fb[1]);
    stage(r + 1, fa[1], fb[1], fa[0], fb[0]);
  }
  const unsigned long long t1 = clock64(), w1 = wall_clock64();
  int32_t s = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) s += acc[a][c][v];
  out[blockIdx.x * 256 + tid] = s;
  if (tid == 0) {
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = w1 - w0;
  }
}

int launch_probe(int variant, int rounds, int blocks, int32_t *out, unsigned long long *clk,
                 hipStream_t s) {
  const uint32_t seed = 0x2545f491u;
  if (variant == 0)
    hipLaunchKernelGGL(k_mfma_probe<0>, dim3(blocks), dim3(256), 0, s, rounds, seed, out, clk);
  else if (variant == 1)
    hipLaunchKernelGGL(k_mfma_probe<1>, dim3(blocks), dim3(256), 0, s, rounds, seed, out, clk);
  else
    hipLaunchKernelGGL(k_mfma_probe<2>, dim3(blocks), dim3(256), 0, s, rounds, seed, out, clk);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

extern "C" int refeig_mfma_ceiling(int variant, double seconds, refeig_stream_t stream,
                                   double *ms, double *pops, double *ghz) {
  if (variant < 0 || variant > 2 || !(seconds > 0.0) || seconds > 10.0 || !ms || !pops || !ghz)
    return REFEIG_E_ARG;
  int dev = 0, cus = 0, wall_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      cus <= 0 || wall_khz <= 0)
    return REFEIG_E_HIP;
  hipStream_t s = (hipStream_t)stream;
  const int blocks = cus;
  int32_t *out = nullptr;
  unsigned long long *clk = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = REFEIG_E_HIP;
  std::vector<unsigned long long> hclk(2 * blocks);
  if (hipMalloc(&out, sizeof(int32_t) * 256 * blocks) != hipSuccess) return REFEIG_E_NOMEM;
  if (hipMalloc(&clk, sizeof(unsigned long long) * 2 * blocks) != hipSuccess) {
    (void)hipFree(out);
    return REFEIG_E_NOMEM;
  }
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    // calibrate on a short run, then time runs of about `seconds`, keeping the last
    int rounds = 1024;
    float t = 0.0f;
    bool ok = true;
    for (int pass = 0; pass < 4 && ok; ++pass) {
      ok = hipEventRecord(e0, s) == hipSuccess &&
           launch_probe(variant, rounds, blocks, out, clk, s) == 0 &&
           hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&t, e0, e1) == hipSuccess;
      if (ok && pass == 0) {
        double r = rounds * (seconds * 1e3 / (t > 0.05f ? t : 0.05f));
        r = r < 2.0 ? 2.0 : r > (double)(1 << 24) ? (double)(1 << 24) : r;
        rounds = ((int)r + 1) & ~1;
      }
    }
    ok = ok && hipMemcpy(hclk.data(), clk, sizeof(unsigned long long) * 2 * blocks,
                         hipMemcpyDeviceToHost) == hipSuccess;
    if (ok) {
      double cyc = 0.0, wall = 0.0;
      for (int b = 0; b < blocks; ++b) {
        cyc += (double)hclk[2 * b];
        wall += (double)hclk[2 * b + 1];
      }
      // per stage and block: 4 waves x 32 MFMAs x 32 x 32 x 32 multiply-adds x 2
      const double ops = (double)blocks * rounds * 4.0 * 32.0 * 65536.0;
      *ms = t;
      *pops = ops / (t * 1e-3) / 1e15;
      *ghz = wall > 0.0 ? cyc / (wall / (wall_khz * 1e3)) / 1e9 : 0.0;
      st = REFEIG_OK;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  (void)hipFree(clk);
  return st;
}
