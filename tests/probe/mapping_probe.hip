// mapping_probe.hip -- two mappings of the per-block work up to bit-plane
// formation, on the same blocks: block exponent, block-floating-point cast,
// forward lifting, sequency order, negabinary, and the 32 bit planes of the
// 64 coefficients (the steps of the paper's Section II-C codec before the
// embedded coder).
//   lane: one block per lane, 64 blocks per wavefront -- the library's
//         mapping, built from the library's own block code; planes by the
//         64x32 SWAR bit transpose;
//   wave: one block per wavefront and one value per lane, lifting through
//         lane shuffles, each bit plane one ballot.
// A small run checks that both produce the same plane words; a large run
// (1M blocks, 268 MB of float32) times both.  Built by the package's build
// step; run by tests/test_gpu_mapping_probe.py and under rocprofv3 for the
// instruction counts.  A measurement program, not part of the library.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include <math.h>
#include <vector>
#include "../../paper_2609_24294_amd/csrc/block_codec.hpp"

using namespace zfpx;
#define CHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); return 1; } } while (0)

struct Grid { int nx, ny, nz, nbx, nby, nbz; };

__device__ __forceinline__ uint64_t fold_planes(const uint64_t* P) {
  uint64_t f = 0;
#pragma unroll
  for (int k = 0; k < 32; k++) f ^= (P[k] << k) | (P[k] >> ((64 - k) & 63));
  return f;
}

// one block per lane
template <bool FULL>
__global__ __launch_bounds__(128) void k_lane(Grid g, const float* __restrict__ src, uint64_t* __restrict__ out, int nblocks) {
  const int b = blockIdx.x * 128 + threadIdx.x;
  if (b >= nblocks) return;
  const int bx = b % g.nbx, by = (b / g.nbx) % g.nby, bz = b / (g.nbx * g.nby);
  float v[64];
#pragma unroll
  for (int z = 0; z < 4; z++)
#pragma unroll
    for (int y = 0; y < 4; y++) {
      const float4 f = *reinterpret_cast<const float4*>(src + ((size_t)(4 * bz + z) * g.ny + 4 * by + y) * g.nx + 4 * bx);
      v[16 * z + 4 * y + 0] = f.x; v[16 * z + 4 * y + 1] = f.y; v[16 * z + 4 * y + 2] = f.z; v[16 * z + 4 * y + 3] = f.w;
    }
  float amax = 0.0f;
#pragma unroll
  for (int i = 0; i < 64; i++) amax = __builtin_fmaxf(amax, __builtin_fabsf(v[i]));
  const int emax = (int)(f32_bits(amax) >> 23) - 126;
  const float sc = scale_pow2(1.0f, 30 - emax);
  int32_t q[64];
#pragma unroll
  for (int i = 0; i < 64; i++) q[i] = (int32_t)(v[i] * sc);
  xform_fwd(q);
  uint64_t X[32];
#pragma unroll
  for (int s = 0; s < 32; s++)
    X[s] = (uint64_t)((uint32_t)q[kSeq.idx[s]] + kNegabinaryMask) |
           ((uint64_t)((uint32_t)q[kSeq.idx[32 + s]] + kNegabinaryMask) << 32);
  transpose32x2<true>(X);
  if (FULL) {
    for (int k = 0; k < 32; k++) out[(size_t)b * 32 + k] = X[k];
  } else {
    out[b] = fold_planes(X);
  }
}

// one block per wavefront (grid-stride over blocks)
__device__ __forceinline__ void lift4(int32_t& x0, int32_t& x1, int32_t& x2, int32_t& x3) { lift_fwd(x0, x1, x2, x3); }
__device__ __forceinline__ int32_t pick(int j, int32_t a0, int32_t a1, int32_t a2, int32_t a3) {
  return j == 0 ? a0 : j == 1 ? a1 : j == 2 ? a2 : a3;
}

template <bool FULL>
__global__ __launch_bounds__(256) void k_wave(Grid g, const float* __restrict__ src, uint64_t* __restrict__ out, int nblocks) {
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * 4;
  const int x = lane & 3, y = (lane >> 2) & 3, z = lane >> 4;
  const int sidx = kSeq.idx[lane];
  for (int b = blockIdx.x * 4 + (threadIdx.x >> 6); b < nblocks; b += waves) {
    const int bx = b % g.nbx, by = (b / g.nbx) % g.nby, bz = b / (g.nbx * g.nby);
    const float v = src[((size_t)(4 * bz + z) * g.ny + 4 * by + y) * g.nx + 4 * bx + x];
    float m = __builtin_fabsf(v);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = __builtin_fmaxf(m, __shfl_xor(m, o, 64));
    const int emax = (int)(f32_bits(m) >> 23) - 126;
    int32_t q = (int32_t)(v * scale_pow2(1.0f, 30 - emax));
    {  // x-lines
      const int base = lane & ~3;
      int32_t a0 = __shfl(q, base, 64), a1 = __shfl(q, base | 1, 64), a2 = __shfl(q, base | 2, 64), a3 = __shfl(q, base | 3, 64);
      lift4(a0, a1, a2, a3);
      q = pick(x, a0, a1, a2, a3);
    }
    {  // y-lines
      const int base = lane & ~12;
      int32_t a0 = __shfl(q, base, 64), a1 = __shfl(q, base | 4, 64), a2 = __shfl(q, base | 8, 64), a3 = __shfl(q, base | 12, 64);
      lift4(a0, a1, a2, a3);
      q = pick(y, a0, a1, a2, a3);
    }
    {  // z-lines
      const int base = lane & 15;
      int32_t a0 = __shfl(q, base, 64), a1 = __shfl(q, base | 16, 64), a2 = __shfl(q, base | 32, 64), a3 = __shfl(q, base | 48, 64);
      lift4(a0, a1, a2, a3);
      q = pick(z, a0, a1, a2, a3);
    }
    const uint32_t u = ((uint32_t)__shfl(q, sidx, 64) + kNegabinaryMask) ^ kNegabinaryMask;
    uint64_t P[32];
#pragma unroll
    for (int k = 0; k < 32; k++) P[k] = __ballot((u >> k) & 1);
    if (FULL) {
      if (lane < 32) {
        uint64_t mine = 0;
#pragma unroll
        for (int k = 0; k < 32; k++) mine = lane == k ? P[k] : mine;
        out[(size_t)b * 32 + lane] = mine;
      }
    } else {
      const uint64_t f = fold_planes(P);
      if (lane == 0) out[b] = f;
    }
  }
}

int main(int argc, char** argv) {
  int cus = 0;
  CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0)); CHK(hipEventCreate(&e1));
  for (int pass = 0; pass < 2; pass++) {
    const bool check = pass == 0;
    Grid g;
    g.nz = check ? 8 : 64; g.ny = check ? 32 : 256; g.nx = check ? 256 : 4096;
    g.nbx = g.nx / 4; g.nby = g.ny / 4; g.nbz = g.nz / 4;
    const int nblocks = g.nbx * g.nby * g.nbz;
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    std::vector<float> h(n);
    uint64_t s = 12345;
    for (size_t i = 0; i < n; i++) {
      s = s * 6364136223846793005ull + 1442695040888963407ull;
      const double r = (double)(s >> 11) / 9007199254740992.0;
      const size_t xx = i % g.nx, yy = (i / g.nx) % g.ny, zz = i / ((size_t)g.nx * g.ny);
      h[i] = (float)(280.0 + 15.0 * sin(0.01 * xx + 0.03 * yy) * cos(0.05 * zz) + 0.01 * (r - 0.5));
    }
    float* d_src; uint64_t *d_a, *d_b;
    const size_t words = check ? (size_t)nblocks * 32 : (size_t)nblocks;
    CHK(hipMalloc(&d_src, n * 4)); CHK(hipMalloc(&d_a, words * 8)); CHK(hipMalloc(&d_b, words * 8));
    CHK(hipMemcpy(d_src, h.data(), n * 4, hipMemcpyHostToDevice));
    CHK(hipMemset(d_a, 0, words * 8)); CHK(hipMemset(d_b, 0xff, words * 8));
    const int grid_lane = (nblocks + 127) / 128;
    int grid_wave = cus * 8;
    if (grid_wave * 4 > nblocks) grid_wave = (nblocks + 3) / 4;
    if (check) {
      hipLaunchKernelGGL(k_lane<true>, dim3(grid_lane), dim3(128), 0, 0, g, d_src, d_a, nblocks);
      hipLaunchKernelGGL(k_wave<true>, dim3(grid_wave), dim3(256), 0, 0, g, d_src, d_b, nblocks);
      CHK(hipGetLastError()); CHK(hipDeviceSynchronize());
      std::vector<uint64_t> a(words), b(words);
      CHK(hipMemcpy(a.data(), d_a, words * 8, hipMemcpyDeviceToHost));
      CHK(hipMemcpy(b.data(), d_b, words * 8, hipMemcpyDeviceToHost));
      size_t bad = 0;
      for (size_t i = 0; i < words; i++) bad += a[i] != b[i];
      printf("check: %d blocks, %zu of %zu plane words differ\n", nblocks, bad, words);
      if (bad) return 2;
    } else {
      float best_l = 1e30f, best_w = 1e30f;
      for (int rep = 0; rep < 10; rep++) {
        float ms;
        CHK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(k_lane<false>, dim3(grid_lane), dim3(128), 0, 0, g, d_src, d_a, nblocks);
        CHK(hipEventRecord(e1, 0)); CHK(hipEventSynchronize(e1)); CHK(hipEventElapsedTime(&ms, e0, e1));
        if (rep >= 2 && ms < best_l) best_l = ms;
        CHK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(k_wave<false>, dim3(grid_wave), dim3(256), 0, 0, g, d_src, d_b, nblocks);
        CHK(hipEventRecord(e1, 0)); CHK(hipEventSynchronize(e1)); CHK(hipEventElapsedTime(&ms, e0, e1));
        if (rep >= 2 && ms < best_w) best_w = ms;
      }
      CHK(hipGetLastError());
      std::vector<uint64_t> a(words), b(words);
      CHK(hipMemcpy(a.data(), d_a, words * 8, hipMemcpyDeviceToHost));
      CHK(hipMemcpy(b.data(), d_b, words * 8, hipMemcpyDeviceToHost));
      size_t bad = 0;
      for (size_t i = 0; i < words; i++) bad += a[i] != b[i];
      printf("timing: %d blocks (%.1f MB of float32); folds differing: %zu\n", nblocks, n * 4 / 1e6, bad);
      printf("  lane per block: %.4f ms = %.1f ns per 64 blocks\n", best_l, best_l * 1e6 / (nblocks / 64.0));
      printf("  wave per block: %.4f ms = %.1f ns per 64 blocks (%.2fx)\n", best_w, best_w * 1e6 / (nblocks / 64.0), best_w / best_l);
    }
    CHK(hipFree(d_src)); CHK(hipFree(d_a)); CHK(hipFree(d_b));
  }
  return 0;
}
