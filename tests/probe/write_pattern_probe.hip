// Write-pattern probe for the fixed-rate decoder's stores.
//
// Each 64-thread workgroup reads 16 KB contiguously (a rate-16 tile's stream
// is 8 KB; the read side only has to keep the chip busy) and writes 16 pieces
// of 1 KB: piece p of each of 16 row streams, as a decoded tile writes 4 rows
// of 4 levels, each 1 KB from 64 lanes of 16 bytes.  The row streams start
// either on a 128-byte line or 16 bytes past one (the reduced grid's rows
// start at 16-byte multiples, so a tile's row pieces straddle lines shared
// with the neighbouring tile), and pieces are taken in plain order (the
// neighbour on another XCD) or in the decoder's XCD-grouped order (8
// consecutive pieces per XCD in every group of 64 workgroups).  Prints the
// mean time of 10 launches per variant, two passes.  A last set of variants
// has each workgroup write a run of K consecutive pieces one after another,
// so that the two halves of every shared line but the run's ends come from
// the same wavefront back to back.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

typedef float f4v __attribute__((ext_vector_type(4)));

#define CK(x)                                                            \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                          \
    }                                                                    \
  } while (0)

// npieces is a multiple of 64, so the grouped order is a permutation.
template <bool XCD>
__global__ __launch_bounds__(64) void k_pieces(const f4v* __restrict__ src, float* __restrict__ dst,
                                               size_t row_len, int shift) {
  const unsigned b = blockIdx.x;
  unsigned p = b;
  if (XCD) {
    const unsigned r = b % 64;
    p = (b - r) + (r % 8) * 8 + r / 8;
  }
  const int lane = threadIdx.x;
  f4v v[16];
#pragma unroll
  for (int j = 0; j < 16; j++) v[j] = src[(size_t)p * 1024 + j * 64 + lane];
#pragma unroll
  for (int j = 0; j < 16; j++)
    *reinterpret_cast<f4v*>(dst + (size_t)j * row_len + shift + (size_t)p * 256 + lane * 4) = v[j];
}

// Runs of K consecutive pieces per workgroup (npieces is a multiple of K).
template <int K>
__global__ __launch_bounds__(64) void k_runs(const f4v* __restrict__ src, float* __restrict__ dst,
                                             size_t row_len, int shift) {
  const int lane = threadIdx.x;
  for (int k = 0; k < K; k++) {
    const size_t p = (size_t)blockIdx.x * K + k;
    f4v v[16];
#pragma unroll
    for (int j = 0; j < 16; j++) v[j] = src[p * 1024 + j * 64 + lane];
#pragma unroll
    for (int j = 0; j < 16; j++)
      *reinterpret_cast<f4v*>(dst + (size_t)j * row_len + shift + p * 256 + lane * 4) = v[j];
  }
}

int main() {
  const unsigned np = 1u << 18;                     // 262,144 pieces: 4 GiB read, 4 GiB written
  const size_t row_len = (size_t)np * 256 + 64;      // floats per row stream, room for a shift
  f4v* src;
  float* dst;
  CK(hipMalloc(&src, (size_t)np * 16384));
  CK(hipMalloc(&dst, 16 * row_len * sizeof(float)));
  CK(hipMemset(src, 0x3f, (size_t)np * 16384));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const int shifts[3] = {0, 4, 32};  // floats: on a line, 16 B past one, the next line
  for (int pass = 0; pass < 2; pass++)
    for (int grouped = 0; grouped < 2; grouped++)
      for (int si = 0; si < 3; si++) {
        float total = 0;
        const int reps = 10;
        for (int r = 0; r < reps + 2; r++) {
          CK(hipEventRecord(e0, 0));
          if (grouped)
            hipLaunchKernelGGL(k_pieces<true>, dim3(np), dim3(64), 0, 0, src, dst, row_len,
                               shifts[si]);
          else
            hipLaunchKernelGGL(k_pieces<false>, dim3(np), dim3(64), 0, 0, src, dst, row_len,
                               shifts[si]);
          CK(hipGetLastError());
          CK(hipEventRecord(e1, 0));
          CK(hipEventSynchronize(e1));
          float ms;
          CK(hipEventElapsedTime(&ms, e0, e1));
          if (r >= 2) total += ms;
        }
        const double ms = total / reps, bytes = 2.0 * np * 16384.0;
        printf("pass %d order=%s row start %3d B past a line: %.4f ms  %.1f GB/s  %.1f%% of 8 TB/s\n",
               pass, grouped ? "xcd-grouped" : "plain      ", (shifts[si] * 4) % 128, ms,
               bytes / ms / 1e6, bytes / ms / 1e6 / 80.0);
        fflush(stdout);
      }
  for (int pass = 0; pass < 2; pass++)
    for (int K : {4, 16})
      for (int si = 0; si < 2; si++) {
        float total = 0;
        const int reps = 10;
        for (int r = 0; r < reps + 2; r++) {
          CK(hipEventRecord(e0, 0));
          if (K == 4)
            hipLaunchKernelGGL(k_runs<4>, dim3(np / 4), dim3(64), 0, 0, src, dst, row_len,
                               shifts[si]);
          else
            hipLaunchKernelGGL(k_runs<16>, dim3(np / 16), dim3(64), 0, 0, src, dst, row_len,
                               shifts[si]);
          CK(hipGetLastError());
          CK(hipEventRecord(e1, 0));
          CK(hipEventSynchronize(e1));
          float ms;
          CK(hipEventElapsedTime(&ms, e0, e1));
          if (r >= 2) total += ms;
        }
        const double ms = total / reps, bytes = 2.0 * np * 16384.0;
        printf("pass %d runs of %2d pieces   row start %3d B past a line: %.4f ms  %.1f GB/s  %.1f%% of 8 TB/s\n",
               pass, K, shifts[si] * 4, ms, bytes / ms / 1e6, bytes / ms / 1e6 / 80.0);
        fflush(stdout);
      }
  CK(hipFree(src));
  CK(hipFree(dst));
  return 0;
}
