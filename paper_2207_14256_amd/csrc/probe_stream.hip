// Streaming ceiling of one MI355X for the push's access pattern: a plain
// kernel that reads nine and writes six 4-byte arrays per element (36 B in,
// 24 B out, as the FP32 push's particle state), and a 16-byte copy, each with
// ordinary and with non-temporal accesses.  It bounds what a push could reach
// with a perfectly cached mesh.  Standalone executable (built next to the
// library); prints one line per timed case.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);  \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

namespace {

struct Pattern {
  const float* in[9];
  float* out[6];
  long n;
};

template <bool NT>
__global__ void __launch_bounds__(256) k_pattern(Pattern p) {
  const long i = blockIdx.x * 256L + threadIdx.x;
  if (i >= p.n) return;
  float v[9];
  for (int k = 0; k < 9; ++k) v[k] = NT ? __builtin_nontemporal_load(&p.in[k][i]) : p.in[k][i];
  for (int k = 0; k < 6; ++k) {
    const float r = v[k] + v[(k + 3) % 9] * 0.5f;
    if (NT) __builtin_nontemporal_store(r, &p.out[k][i]);
    else p.out[k][i] = r;
  }
}

typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void __launch_bounds__(256) k_copy16(const v4f* a, v4f* b, long n) {
  const long i = blockIdx.x * 256L + threadIdx.x;
  if (i >= n) return;
  if (NT) __builtin_nontemporal_store(__builtin_nontemporal_load(&a[i]), &b[i]);
  else b[i] = a[i];
}

}  // namespace

int main() {
  const long n = 134217728;   // 512^3 elements
  std::vector<float*> bufs(15);
  for (auto& b : bufs) {
    CHECK(hipMalloc(&b, n * 4));
    CHECK(hipMemset(b, 0, n * 4));
  }
  Pattern p;
  for (int k = 0; k < 9; ++k) p.in[k] = bufs[k];
  for (int k = 0; k < 6; ++k) p.out[k] = bufs[9 + k];
  p.n = n;
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const unsigned nb = (unsigned)((n + 255) / 256);
  for (int nt = 0; nt < 2; ++nt) {
    for (int rep = 0; rep < 3; ++rep) {
      CHECK(hipEventRecord(e0));
      for (int it = 0; it < 10; ++it) {
        if (nt) hipLaunchKernelGGL(k_pattern<true>, dim3(nb), dim3(256), 0, 0, p);
        else hipLaunchKernelGGL(k_pattern<false>, dim3(nb), dim3(256), 0, 0, p);
      }
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      ms /= 10;
      std::printf("push pattern (36 B read + 24 B write per element, n = %ld) nontemporal=%d: %.3f ms, %.2f TB/s\n",
                  n, nt, ms, 60.0 * n / ms / 1e9);
    }
  }
  for (auto& b : bufs) CHECK(hipFree(b));
  const long bytes = 1L << 32;
  v4f *a, *b;
  CHECK(hipMalloc(&a, bytes));
  CHECK(hipMalloc(&b, bytes));
  CHECK(hipMemset(a, 0, bytes));
  const long n16 = bytes / 16;
  const unsigned nb16 = (unsigned)((n16 + 255) / 256);
  for (int nt = 0; nt < 2; ++nt) {
    for (int rep = 0; rep < 3; ++rep) {
      CHECK(hipEventRecord(e0));
      for (int it = 0; it < 10; ++it) {
        if (nt) hipLaunchKernelGGL(k_copy16<true>, dim3(nb16), dim3(256), 0, 0, a, b, n16);
        else hipLaunchKernelGGL(k_copy16<false>, dim3(nb16), dim3(256), 0, 0, a, b, n16);
      }
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      ms /= 10;
      std::printf("copy 4 GiB, 16 B per thread, nontemporal=%d: %.3f ms, %.2f TB/s (read + write)\n", nt, ms,
                  2.0 * bytes / ms / 1e9);
    }
  }
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  CHECK(hipDeviceSynchronize());
  return 0;
}
