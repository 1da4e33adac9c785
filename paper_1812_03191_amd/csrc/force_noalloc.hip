// force_noalloc.hip -- the force of eq. 18 over a caller's density field with
// no device allocation: the per-block partials live in a file-scope device
// array (`scratch`), one per GPU for the life of the process.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  Its
// allocating counterpart is df_force, whose partials sit in the run's arena.
#include <cmath>
#include <mutex>

#include "df.h"
#include "dfk.h"

// raises an error on the calling thread (api.hip)
int df_fail_internal(int code, const char *msg);

namespace {

constexpr int NF_THREADS = 256;
constexpr int NF_MAXBLOCKS = 4096;  // partial slots per plane: scratch holds 3 * 4096 doubles (96 KiB)
constexpr int NF_MAXDEV = 64;

// per-block partials of the three force components, three planes of
// NF_MAXBLOCKS values; each launch writes every slot it later reads
static __device__ __align__(256) double scratch[3 * NF_MAXBLOCKS];

// device address of `scratch` on each GPU (the name itself is a host-side
// stand-in and must never reach a kernel)
double *g_ptr[NF_MAXDEV];
int g_rc[NF_MAXDEV];
std::once_flag g_once[NF_MAXDEV];

int scratch_of_current_device(double **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NF_MAXDEV)
    return df_fail_internal(DF_EDEVICE, "df_force_density: no current HIP device");
  std::call_once(g_once[dev], [dev] {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_rc[dev] = (e == hipSuccess && p) ? DF_OK : DF_EDEVICE;
    g_ptr[dev] = static_cast<double *>(p);
  });
  if (g_rc[dev]) return df_fail_internal(DF_EDEVICE, "df_force_density: scratch address not available");
  *out = g_ptr[dev];
  return DF_OK;
}

__device__ __forceinline__ double nf_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// fixed-order sum of one value per thread of a 256-thread block (thread 0 gets it)
__device__ __forceinline__ double nf_block_sum(double v, double *sh) {
  v = nf_wave_sum(v);
  const int t = threadIdx.x;
  if (t % 64 == 0) sh[t / 64] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0)
    for (int w = 0; w < NF_THREADS / 64; ++w) s += sh[w];
  __syncthreads();
  return s;
}

struct NfArgs {
  const double *rho;
  int nx, ny, nz;
  double dx, GM, eps2, rho0;
  double *part;  // scratch partials (device address)
  int nb;        // blocks of the launch = partial slots used per plane
};

// Eq. 18 on one level whose central vertex is the perturber: G M (rho - rho0)
// dx^3 r / (r^2 + eps^2)^{3/2} per cell, r the cell centre; each block sums a
// grid-stride share of the cells and writes its three partials.
__global__ void __launch_bounds__(NF_THREADS) k_nf_partials(NfArgs A) {
  __shared__ double sh[NF_THREADS / 64];
  const long n = (long)A.nx * A.ny * A.nz;
  const double vol = A.dx * A.dx * A.dx;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for (long c = (long)blockIdx.x * NF_THREADS + threadIdx.x; c < n; c += (long)A.nb * NF_THREADS) {
    const int i = (int)(c % A.nx);
    const long r = c / A.nx;
    const int j = (int)(r % A.ny), k = (int)(r / A.ny);
    const double x = ((double)i - 0.5 * A.nx + 0.5) * A.dx;
    const double y = ((double)j - 0.5 * A.ny + 0.5) * A.dx;
    const double z = ((double)k - 0.5 * A.nz + 0.5) * A.dx;
    const double d2 = x * x + y * y + z * z + A.eps2;
    const double w = A.GM * (A.rho[c] - A.rho0) * vol / (d2 * sqrt(d2));
    fx += w * x;
    fy += w * y;
    fz += w * z;
  }
  const double sx = nf_block_sum(fx, sh), sy = nf_block_sum(fy, sh), sz = nf_block_sum(fz, sh);
  if (threadIdx.x == 0) {
    A.part[blockIdx.x] = sx;
    A.part[NF_MAXBLOCKS + blockIdx.x] = sy;
    A.part[2 * NF_MAXBLOCKS + blockIdx.x] = sz;
  }
}

// one block: the partials summed in a fixed order into out[0..2]
__global__ void __launch_bounds__(NF_THREADS) k_nf_final(const double *part, int nb, double *out) {
  __shared__ double sh[NF_THREADS / 64];
  for (int q = 0; q < 3; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += NF_THREADS) s += part[q * NF_MAXBLOCKS + b];
    s = nf_block_sum(s, sh);
    if (threadIdx.x == 0) out[q] = s;
  }
}

}  // namespace

extern "C" int df_force_density(const double *rho, int32_t nx, int32_t ny, int32_t nz, double dx, double GM,
                                double eps, double rho0, double *out, void *stream) {
  if (!rho || !out) return df_fail_internal(DF_EINVAL, "df_force_density: null pointer");
  if (nx < 2 || ny < 2 || nz < 2 || nx % 2 || ny % 2 || nz % 2)
    return df_fail_internal(DF_EINVAL, "df_force_density: cell counts must be even and >= 2");
  const long n = (long)nx * ny * nz;
  if (n > DF_FORCE_DENSITY_MAX_CELLS)
    return df_fail_internal(DF_EINVAL, "df_force_density: more cells than DF_FORCE_DENSITY_MAX_CELLS");
  if (!(dx > 0.0) || !std::isfinite(dx) || !std::isfinite(GM) || !std::isfinite(eps) || !std::isfinite(rho0) ||
      GM < 0.0 || eps < 0.0)
    return df_fail_internal(DF_EINVAL, "df_force_density: bad dx, GM, eps or rho0");
  double *part = nullptr;
  int rc = scratch_of_current_device(&part);
  if (rc) return rc;
  long nb = (n + NF_THREADS - 1) / NF_THREADS;
  if (nb > NF_MAXBLOCKS) nb = NF_MAXBLOCKS;
  NfArgs A{rho, nx, ny, nz, dx, GM, eps * eps, rho0, part, (int)nb};
  hipStream_t st = (hipStream_t)stream;
  k_nf_partials<<<dim3((unsigned)nb), dim3(NF_THREADS), 0, st>>>(A);
  k_nf_final<<<dim3(1), dim3(NF_THREADS), 0, st>>>(part, (int)nb, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return df_fail_internal(DF_EDEVICE, hipGetErrorString(e));
  return DF_OK;
}
