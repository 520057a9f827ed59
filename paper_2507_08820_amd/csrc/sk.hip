// sk.hip -- shell binning of the static structure factor (arXiv:2507.08820,
// Sec. III: spectra of a normalised FFT averaged over wavevectors of equal
// modulus).
//
// Input: the R2C transform F(n) = sum_x dm(x) exp(-2 pi i n.x / L) of one real
// moment field on an nz x ny x nx box (x fastest), stored as nz x ny x (nx/2+1)
// complex values.  For every stored n != 0, |F(n)|^2 / N is added to shell
// round(|n|) with n_a taken in (-L_a/2, L_a/2].  Only kx = 0..nx/2 is stored;
// the other half of the spectrum is the complex conjugate (real input), so
// every stored column except kx = 0 and kx = nx/2 (nx even) counts twice.
// Shell sums are privatised in LDS per block (FP64) and added to the global
// FP64 sums with one atomic per shell and block.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rflbm {

namespace {

__global__ void sk_bin_kernel(const float2* __restrict__ spec, uint32_t nx, uint32_t ny, uint32_t nz,
                              uint32_t nshells, double inv_n, double* __restrict__ shell_sum,
                              unsigned long long* __restrict__ shell_count) {
  extern __shared__ double lds[];
  double* sum = lds;
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(lds + nshells);
  for (uint32_t s = threadIdx.x; s < nshells; s += blockDim.x) {
    sum[s] = 0.0;
    cnt[s] = 0ull;
  }
  __syncthreads();
  const uint32_t hx = nx / 2 + 1;
  const uint64_t total = static_cast<uint64_t>(hx) * ny * nz;
  for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t kx = static_cast<uint32_t>(e % hx);
    const uint64_t r = e / hx;
    const uint32_t ky = static_cast<uint32_t>(r % ny);
    const uint32_t kz = static_cast<uint32_t>(r / ny);
    const int64_t sx = kx;
    const int64_t sy = ky <= ny / 2 ? static_cast<int64_t>(ky) : static_cast<int64_t>(ky) - ny;
    const int64_t sz = kz <= nz / 2 ? static_cast<int64_t>(kz) : static_cast<int64_t>(kz) - nz;
    const int64_t k2 = sx * sx + sy * sy + sz * sz;
    if (k2 == 0) continue;
    const uint32_t shell = static_cast<uint32_t>(llrint(sqrt(static_cast<double>(k2))));
    if (shell >= nshells) continue;
    const bool self_conj = kx == 0 || (nx % 2 == 0 && kx == nx / 2);
    const unsigned mult = self_conj ? 1u : 2u;
    const float2 c = spec[e];
    const double p = (static_cast<double>(c.x) * c.x + static_cast<double>(c.y) * c.y) * inv_n;
    atomicAdd(&sum[shell], p * mult);
    if (shell_count) atomicAdd(&cnt[shell], static_cast<unsigned long long>(mult));
  }
  __syncthreads();
  for (uint32_t s = threadIdx.x; s < nshells; s += blockDim.x) {
    if (sum[s] != 0.0) atomicAdd(&shell_sum[s], sum[s]);
    if (shell_count && cnt[s]) atomicAdd(&shell_count[s], cnt[s]);
  }
}

}  // namespace

hipError_t launch_sk_bin(const void* spec, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t nshells,
                         double* shell_sum, unsigned long long* shell_count, hipStream_t s) {
  const uint64_t total = static_cast<uint64_t>(nx / 2 + 1) * ny * nz;
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  const size_t lds = static_cast<size_t>(nshells) * (sizeof(double) + sizeof(unsigned long long));
  hipLaunchKernelGGL(sk_bin_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), lds, s,
                     static_cast<const float2*>(spec), nx, ny, nz, nshells,
                     1.0 / (static_cast<double>(nx) * ny * nz), shell_sum, shell_count);
  return hipGetLastError();
}

}  // namespace rflbm
