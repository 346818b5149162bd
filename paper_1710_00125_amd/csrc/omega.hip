// The sketch matrix Omega (Section 3) written out for the factorization and
// for tests; the generator itself is in omega_dev.h.
#include "common.h"
#include "kernels.h"
#include "omega_dev.h"

namespace rcp {
namespace {

using namespace omega_dev;

__global__ void omega_kernel(uint64_t seed, uint64_t stream, int l, int64_t n, double* out,
                             int transposed, int lpad) {
  const int64_t total = (int64_t)l * n;
  const int64_t nctr = (total + 3) / 4;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nctr;
       c += (int64_t)gridDim.x * blockDim.x) {
    double z[4];
    omega_quad(seed, c, z, stream);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t q = 4 * c + t;
      if (q < total) {
        if (!transposed) {
          out[q] = z[t];
        } else {
          const int64_t i = q / n, j = q - i * n;
          out[j * lpad + i] = z[t];
        }
      }
    }
  }
}

__global__ void zero_pad_rows_kernel(double* out, int64_t n, int l, int lpad) {
  const int w = lpad - l;
  const int64_t total = n * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / w;
    out[j * lpad + l + (e - j * w)] = 0.0;
  }
}

}  // namespace

void launch_omega(uint64_t seed, int l, int64_t n, double* out, int transposed, int lpad,
                  hipStream_t s, uint64_t stream) {
  const int64_t nctr = ((int64_t)l * n + 3) / 4;
  if (nctr > 0) {
    const int64_t blocks = std::min<int64_t>((nctr + 255) / 256, 65536);
    hipLaunchKernelGGL(omega_kernel, dim3((unsigned)blocks), dim3(256), 0, s, seed, stream, l, n,
                       out, transposed, lpad);
  }
  if (transposed && lpad > l && n > 0) {
    const int64_t total = n * (lpad - l);
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(zero_pad_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, n, l,
                       lpad);
  }
}

}  // namespace rcp
