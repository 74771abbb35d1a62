// Rank growing (Sec. III.C): the state added to the ansatz is a random
// special orthogonal transformation Q, close to the identity, applied to a
// state of high amplitude: Gamma' = Q Gamma Q^T.  It runs once per added
// state, so the two products are plain LDS-tiled ones on the vector units.
#include <mutex>

#include "sgs_internal.h"

namespace sgs {

constexpr int RT = 16;

// C = A B (tb = 0) or A B^T (tb = 1); n x n row-major.
// grid: (ceil(n / 16), ceil(n / 16)), 16 x 16 threads
__global__ __launch_bounds__(256) void k_rot_mul(const double* __restrict__ A, const double* __restrict__ B,
                                                 double* __restrict__ C, int n, int tb) {
  __shared__ double As[RT][RT + 1], Bs[RT][RT + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int row = blockIdx.y * RT + ty, col = blockIdx.x * RT + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < n; k0 += RT) {
    As[ty][tx] = (row < n && k0 + tx < n) ? A[(long long)row * n + k0 + tx] : 0.0;
    const int bk = k0 + ty;  // Bs[ty][tx] = B[k0 + ty][col] (or B^T)
    double bv = 0.0;
    if (bk < n && col < n) bv = tb ? B[(long long)col * n + bk] : B[(long long)bk * n + col];
    Bs[ty][tx] = bv;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < RT; ++kk) acc = fma(As[ty][kk], Bs[kk][tx], acc);
    __syncthreads();
  }
  if (row < n && col < n) C[(long long)row * n + col] = acc;
}

// C <- (C - C^T) / 2 in place (each pair (i < j) by one thread)
__global__ __launch_bounds__(256) void k_rot_skew(double* __restrict__ C, int n) {
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (long long)i * n);
    if (i > j) continue;
    if (i == j) {
      C[e] = 0.0;
      continue;
    }
    const long long t = (long long)j * n + i;
    const double v = 0.5 * (C[e] - C[t]);
    C[e] = v;
    C[t] = -v;
  }
}

// Scratch of the allocation-free variant: the intermediate Q Gamma for
// n <= ROTATE_SCRATCH_N.  Each device holds its own copy for the life of the
// process; host code reaches it only through the address hipGetSymbolAddress
// returns on that device (the array's name is not a device address on the host).
__device__ __align__(256) double scratch[ROTATE_SCRATCH_N * ROTATE_SCRATCH_N];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t rotate_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = (double*)p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_rotate(const double* Q, const double* G, double* work, double* out, int n, hipStream_t s) {
  const dim3 grid((n + RT - 1) / RT, (n + RT - 1) / RT), block(RT, RT);
  hipLaunchKernelGGL(k_rot_mul, grid, block, 0, s, Q, G, work, n, 0);
  hipLaunchKernelGGL(k_rot_mul, grid, block, 0, s, (const double*)work, Q, out, n, 1);
  long long b = ((long long)n * n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_rot_skew, dim3((int)b), dim3(256), 0, s, out, n);
  return hipGetLastError();
}

}  // namespace sgs
