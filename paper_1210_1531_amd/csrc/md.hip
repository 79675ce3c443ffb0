// Elementwise pieces of one MD step (velocity Verlet) and a deterministic sum.
//
// An MD step of the method rebuilds H and S at the new structure, solves the
// columns, and takes energy and forces through the density matrix; the time
// step itself is the cheap part and runs here, on the same stream, so the
// positions and velocities stay in device memory across steps.
#include "mag_internal.h"

namespace mag {

// one amu * (Angstrom / fs)^2 in eV: 1.66053906660e-27 kg * 1e10 m^2 s^-2
// over 1.602176634e-19 J (CODATA 2018)
const double AMU_A2_FS2_EV = 1.66053906660e-17 / 1.602176634e-19;

constexpr int MTPB = 256;
constexpr int SUM_TPB = 1024;

static unsigned grid_for(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

__global__ void md_kick_kernel(double* v, const double* F, int64_t n3, double c) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n3) v[i] = fma(c, F[i], v[i]);
}

// x += dt v, then back into [0, L) per axis
__global__ void md_drift_kernel(double* x, const double* v, int64_t n, double dt, double L0,
                                double L1, double L2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double L[3] = {L0, L1, L2};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double y = x[3 * i + d] + dt * v[3 * i + d];
    x[3 * i + d] = y - L[d] * floor(y / L[d]);
  }
}

__global__ void axpy_kernel(double* y, const double* x, int64_t n, double a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = fma(a, x[i], y[i]);
}

// one workgroup: strided partial sums in a fixed order, then a tree in LDS
__global__ __launch_bounds__(SUM_TPB) void sum_kernel(const double* a, int64_t n, int squares,
                                                       double* out) {
  __shared__ double s[SUM_TPB];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += SUM_TPB) {
    const double x = a[i];
    acc += squares ? x * x : x;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = SUM_TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

hipError_t launch_md_kick(double* v, const double* F, int64_t n3, double c, hipStream_t s) {
  if (n3 <= 0) return hipSuccess;
  hipLaunchKernelGGL(md_kick_kernel, dim3(grid_for(n3, MTPB)), dim3(MTPB), 0, s, v, F, n3, c);
  return hipGetLastError();
}

hipError_t launch_md_drift(double* x, const double* v, int64_t n, double dt, const double cell[3],
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(md_drift_kernel, dim3(grid_for(n, MTPB)), dim3(MTPB), 0, s, x, v, n, dt,
                     cell[0], cell[1], cell[2]);
  return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, int64_t n, double a, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(n, MTPB)), dim3(MTPB), 0, s, y, x, n, a);
  return hipGetLastError();
}

hipError_t launch_sum(const double* a, int64_t n, int squares, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(SUM_TPB), 0, s, a, n, squares, out);
  return hipGetLastError();
}

}  // namespace mag
