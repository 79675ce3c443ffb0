// Chemical potential by bisection and the energy sums (between the two
// Green's-function passes of the memory-saving workflow, Eq. 3).
//
// N(mu) = sum_jk w_jk f((eps_jk - mu)/kT) over the valid Ritz pairs
// (k < nu_eff[j]).  Plain bisection halves [lo, hi] at mid = lo + (hi - lo)/2
// and keeps the upper half when N(mid) < N_e.  To cut the number of grid-wide
// reductions, each launch evaluates N at all 31 midpoints of the next five
// halvings (the binary tree of intervals below the current bracket, each node's
// midpoint formed exactly as plain bisection would) and then walks the tree
// with the plain rule; the result is the same sequence of brackets as plain
// bisection, five levels per launch.  Reductions are deterministic: fixed
// grid-stride partition, fixed in-block order, and the last block to finish
// sums the per-block partials in block order.
#include "mag_internal.h"
#include "wave.h"

namespace mag {

constexpr int MTPB = 256;
constexpr int MLEV = 5;
constexpr int MPTS = (1 << MLEV) - 1;  // 31

int mu_points_per_round() { return MPTS; }
int mu_levels_per_round() { return MLEV; }

__device__ __forceinline__ double fermi_mu(double x) {
  if (x > 0.0) {
    const double e = exp(-x);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + exp(x));
}

// s(f) = -[f ln f + (1-f) ln(1-f)] with f = f(x), 1 - f = f(-x) and
// ln f = -ln(1 + e^x), ln(1 - f) = -ln(1 + e^-x), each via log1p(e^-|x|).
__device__ __forceinline__ double entropy_mu(double x) {
  const double f = fermi_mu(x), g = fermi_mu(-x);
  const double lse = log1p(exp(-fabs(x)));
  const double lnf = -(fmax(x, 0.0) + lse);
  const double lng = -(fmax(-x, 0.0) + lse);
  return -(f * lnf + g * lng);
}

__device__ __forceinline__ double wmin(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = fmin(x, __shfl_xor(x, off));
  return x;
}
__device__ __forceinline__ double wmax(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off));
  return x;
}

// returns true in every thread of the block that finished last
__device__ __forceinline__ bool last_block(MuState* st) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned t = atomicAdd(&st->counter, 1u);
    s_last = (t == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last != 0;
}

__global__ __launch_bounds__(MTPB) void mu_init_kernel(const double* eps, const double* w,
                                                       const int32_t* nu_eff, int64_t M, int nu,
                                                       MuState* st, double* partials) {
  __shared__ double s_r[3][MTPB / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double mn = INFINITY, mx = -INFINITY, bad = 0.0;
  const int64_t total = M * nu;
  for (int64_t idx = blockIdx.x * (int64_t)MTPB + tid; idx < total;
       idx += (int64_t)gridDim.x * MTPB) {
    const int64_t j = idx / nu;
    const int k = (int)(idx - j * nu);
    if (k < nu_eff[j]) {
      const double e = eps[idx], ww = w[idx];
      if (!isfinite(e) || !isfinite(ww)) bad = 1.0;
      mn = fmin(mn, e);
      mx = fmax(mx, e);
    }
  }
  mn = wmin(mn);
  mx = wmax(mx);
  bad = wmax(bad);
  if (lane == 0) {
    s_r[0][wv] = mn;
    s_r[1][wv] = mx;
    s_r[2][wv] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    double a = s_r[0][0], b = s_r[1][0], c = s_r[2][0];
    for (int q = 1; q < MTPB / 64; ++q) {
      a = fmin(a, s_r[0][q]);
      b = fmax(b, s_r[1][q]);
      c = fmax(c, s_r[2][q]);
    }
    partials[3 * blockIdx.x] = a;
    partials[3 * blockIdx.x + 1] = b;
    partials[3 * blockIdx.x + 2] = c;
  }
  if (last_block(st) && tid == 0) {
    double a = INFINITY, b = -INFINITY, c = 0.0;
    for (unsigned q = 0; q < gridDim.x; ++q) {
      a = fmin(a, partials[3 * q]);
      b = fmax(b, partials[3 * q + 1]);
      c = fmax(c, partials[3 * q + 2]);
    }
    st->emin = a;
    st->emax = b;
    st->lo = a - 40.0 * st->kT;
    st->hi = b + 40.0 * st->kT;
    st->levels = 0;
    st->done = 0;
    if (c != 0.0 || !(a <= b)) st->err |= KERR_NONFINITE;
    if (!(st->hi - st->lo > st->tol)) st->done = 1;
    st->mu = st->lo + (st->hi - st->lo) / 2.0;
    st->counter = 0;
  }
}

__global__ __launch_bounds__(MTPB) void mu_round_kernel(const double* eps, const double* w,
                                                        const int32_t* nu_eff, int64_t M, int nu,
                                                        MuState* st, double* partials) {
  __shared__ double s_pts[32];
  __shared__ double s_red[MTPB / 64][32];
  __shared__ double s_N[32];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (st->done) return;  // the same value in every block of this launch
  const double lo0 = st->lo, hi0 = st->hi, kT = st->kT;
  if (tid < MPTS) {
    // node n = tid + 1 of the interval tree: walk from the root
    const int n = tid + 1;
    const int depth = 31 - __clz(n);
    double a = lo0, b = hi0;
    for (int bit = depth - 1; bit >= 0; --bit) {
      const double mid = a + (b - a) / 2.0;
      if ((n >> bit) & 1) a = mid;
      else b = mid;
    }
    s_pts[tid] = a + (b - a) / 2.0;
  } else if (tid == MPTS) {
    s_pts[tid] = 0.0;
  }
  __syncthreads();
  double acc[32];
#pragma unroll
  for (int p = 0; p < 32; ++p) acc[p] = 0.0;
  const int64_t total = M * nu;
  for (int64_t idx = blockIdx.x * (int64_t)MTPB + tid; idx < total;
       idx += (int64_t)gridDim.x * MTPB) {
    const int64_t j = idx / nu;
    const int k = (int)(idx - j * nu);
    if (k < nu_eff[j]) {
      const double e = eps[idx], ww = w[idx];
#pragma unroll
      for (int p = 0; p < MPTS; ++p) acc[p] = fma(ww, fermi_mu((e - s_pts[p]) / kT), acc[p]);
    }
  }
  reduce32(acc);  // acc[t] = total of point 16 b5 + 8 b4 + t
  if ((lane & 15) == 0) {
    const int base = ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8;
#pragma unroll
    for (int t = 0; t < 8; ++t) s_red[wv][base + t] = acc[t];
  }
  __syncthreads();
  if (tid < 32) {
    double t = s_red[0][tid];
    for (int q = 1; q < MTPB / 64; ++q) t += s_red[q][tid];
    partials[32 * blockIdx.x + tid] = t;
  }
  if (last_block(st)) {
    if (tid < 32) {
      double t = 0.0;
      for (unsigned q = 0; q < gridDim.x; ++q) t += partials[32 * q + tid];
      s_N[tid] = t;
    }
    __syncthreads();
    if (tid == 0) {
      double lo = lo0, hi = hi0;
      int n = 1, lev = st->levels, done = 0;
      const double ne = st->ne, tol = st->tol;
      for (int l = 0; l < MLEV; ++l) {
        if (!(hi - lo > tol)) {
          done = 1;
          break;
        }
        const double mid = lo + (hi - lo) / 2.0;
        if (s_N[n - 1] < ne) {
          lo = mid;
          n = 2 * n + 1;
        } else {
          hi = mid;
          n = 2 * n;
        }
        ++lev;
      }
      if (!(hi - lo > tol)) done = 1;
      st->lo = lo;
      st->hi = hi;
      st->levels = lev;
      st->done = done;
      st->mu = lo + (hi - lo) / 2.0;
      st->counter = 0;
    }
  }
}

__global__ __launch_bounds__(MTPB) void energy_kernel(const double* eps, const double* w,
                                                      const int32_t* nu_eff, int64_t M, int nu,
                                                      MuState* st, double* partials) {
  __shared__ double s_red[MTPB / 64][4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double mu = st->mu, kT = st->kT;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t total = M * nu;
  for (int64_t idx = blockIdx.x * (int64_t)MTPB + tid; idx < total;
       idx += (int64_t)gridDim.x * MTPB) {
    const int64_t j = idx / nu;
    const int k = (int)(idx - j * nu);
    if (k < nu_eff[j]) {
      const double e = eps[idx], ww = w[idx];
      const double x = (e - mu) / kT;
      const double f = fermi_mu(x);
      v[0] = fma(ww * f, e, v[0]);
      v[1] = fma(ww, entropy_mu(x), v[1]);
      v[2] = fma(ww, f, v[2]);
    }
  }
  reduce4(v);  // v[0] = total of value 2 b5 + b4
  if ((lane & 15) == 0) s_red[wv][((lane >> 5) & 1) * 2 + ((lane >> 4) & 1)] = v[0];
  __syncthreads();
  if (tid < 4) {
    double t = s_red[0][tid];
    for (int q = 1; q < MTPB / 64; ++q) t += s_red[q][tid];
    partials[4 * blockIdx.x + tid] = t;
  }
  if (last_block(st) && tid == 0) {
    double E = 0.0, S = 0.0, N = 0.0;
    for (unsigned q = 0; q < gridDim.x; ++q) {
      E += partials[4 * q];
      S += partials[4 * q + 1];
      N += partials[4 * q + 2];
    }
    st->E = E;
    st->S_ent = S;
    st->N = N;
    st->counter = 0;
  }
}

hipError_t launch_mu_init(const double* eps, const double* w, const int32_t* nu_eff, int64_t M,
                          int nu, MuState* st, double* partials, int grid, hipStream_t s) {
  hipLaunchKernelGGL(mu_init_kernel, dim3(grid), dim3(MTPB), 0, s, eps, w, nu_eff, M, nu, st,
                     partials);
  return hipGetLastError();
}
hipError_t launch_mu_round(const double* eps, const double* w, const int32_t* nu_eff, int64_t M,
                           int nu, MuState* st, double* partials, int grid, hipStream_t s) {
  hipLaunchKernelGGL(mu_round_kernel, dim3(grid), dim3(MTPB), 0, s, eps, w, nu_eff, M, nu, st,
                     partials);
  return hipGetLastError();
}
hipError_t launch_energy(const double* eps, const double* w, const int32_t* nu_eff, int64_t M,
                         int nu, MuState* st, double* partials, int grid, hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(grid), dim3(MTPB), 0, s, eps, w, nu_eff, M, nu, st,
                     partials);
  return hipGetLastError();
}

}  // namespace mag
