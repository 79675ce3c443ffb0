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

// walks the valid Ritz terms (j, k < nu_eff[j]) of a grid-stride partition of
// the M x nu table; the column/row pair is advanced without a division per term
template <class F>
__device__ __forceinline__ void for_terms(const double* eps, const double* w,
                                          const int32_t* nu_eff, int64_t M, int nu, F&& f) {
  const int64_t stride = (int64_t)gridDim.x * MTPB;
  int64_t idx = blockIdx.x * (int64_t)MTPB + threadIdx.x;
  if (idx >= M * nu) return;
  int64_t j = idx / nu;
  int k = (int)(idx - j * nu);
  const int64_t sj = stride / nu;
  const int sk = (int)(stride - sj * nu);
  int ne = nu_eff[j];
  for (; j < M;) {
    if (k < ne) f(eps[j * nu + k], w[j * nu + k]);
    j += sj;
    k += sk;
    if (k >= nu) {
      k -= nu;
      ++j;
    }
    if (j < M) ne = nu_eff[j];
  }
}

// Column sums of a rows x ncomp table of per-block partials (row-major), by
// all MTPB threads of the last block: thread t takes component t % ncomp and
// every (MTPB / ncomp)-th row starting at t / ncomp; the slices are then added
// in slice order.  The order is fixed, so the result is reproducible.
// Returns the total of component tid in threads tid < ncomp.
template <class Op>
__device__ __forceinline__ double block_sum_partials(const double* partials, int rows, int ncomp,
                                                     double init, Op op, double* s_tmp) {
  const int tid = threadIdx.x;
  const int nsl = MTPB / ncomp;
  const int c = tid % ncomp, sl = tid / ncomp;
  double a[4] = {init, init, init, init};
  if (sl < nsl) {
    int r = sl;
    for (; r + 3 * nsl < rows; r += 4 * nsl) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = op(a[u], partials[(int64_t)(r + u * nsl) * ncomp + c]);
    }
    for (int u = 0; r < rows; r += nsl, ++u) a[u & 3] = op(a[u & 3], partials[(int64_t)r * ncomp + c]);
    s_tmp[sl * ncomp + c] = op(op(a[0], a[1]), op(a[2], a[3]));
  }
  __syncthreads();
  double t = init;
  if (tid < ncomp)
    for (int q = 0; q < nsl; ++q) t = op(t, s_tmp[q * ncomp + tid]);
  return t;
}
struct OpAdd {
  __device__ double operator()(double x, double y) const { return x + y; }
};
struct OpMin {
  __device__ double operator()(double x, double y) const { return fmin(x, y); }
};
struct OpMax {
  __device__ double operator()(double x, double y) const { return fmax(x, y); }
};

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
  for_terms(eps, w, nu_eff, M, nu, [&](double e, double ww) {
    if (!isfinite(e) || !isfinite(ww)) bad = 1.0;
    mn = fmin(mn, e);
    mx = fmax(mx, e);
  });
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
  if (last_block(st)) {
    __shared__ double s_tmp[MTPB];
    __shared__ double s_res[3];
    const double r0 = block_sum_partials(partials, (int)gridDim.x, 3, INFINITY, OpMin{}, s_tmp);
    if (tid == 0) s_res[0] = r0;
    __syncthreads();
    const double r1 = block_sum_partials(partials, (int)gridDim.x, 3, -INFINITY, OpMax{}, s_tmp);
    if (tid == 1) s_res[1] = r1;
    __syncthreads();
    const double r2 = block_sum_partials(partials, (int)gridDim.x, 3, 0.0, OpMax{}, s_tmp);
    if (tid == 2) s_res[2] = r2;
    __syncthreads();
    if (tid == 0) {
    const double a = s_res[0], b = s_res[1], c = s_res[2];
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
}

__global__ __launch_bounds__(MTPB) void mu_round_kernel(const double* eps, const double* w,
                                                        const int32_t* nu_eff, int64_t M, int nu,
                                                        MuState* st, double* partials) {
  __shared__ double s_pts[32];
  __shared__ double s_cp[32];
  __shared__ double s_red[MTPB / 64][32];
  __shared__ double s_N[32];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (st->done) return;  // the same value in every block of this launch
  const double lo0 = st->lo, hi0 = st->hi, kT = st->kT;
  const double mu0 = lo0 + (hi0 - lo0) / 2.0;
  // with the bracket narrow on the kT scale, f at every point follows from one
  // exponential per term: exp((e - mu_p)/kT) = exp((e - mu0)/kT) exp((mu0 - mu_p)/kT)
  const bool factored = (hi0 - lo0) <= 600.0 * kT;
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
    const double pt = a + (b - a) / 2.0;
    s_pts[tid] = pt;
    s_cp[tid] = exp((mu0 - pt) / kT);
  } else if (tid == MPTS) {
    s_pts[tid] = 0.0;
    s_cp[tid] = 1.0;
  }
  __syncthreads();
  double acc[32];
#pragma unroll
  for (int p = 0; p < 32; ++p) acc[p] = 0.0;
  if (factored) {
    double cp[MPTS];
#pragma unroll
    for (int p = 0; p < MPTS; ++p) cp[p] = s_cp[p];
    for_terms(eps, w, nu_eff, M, nu, [&](double e, double ww) {
      // |mu0 - mu_p| <= 300 kT, so clamping the exponent at 400 changes f only
      // where it is within e^-100 of 0 or 1, and every product stays finite
      const double E = exp(fmin(fmax((e - mu0) / kT, -400.0), 400.0));
#pragma unroll
      for (int p = 0; p < MPTS; ++p) {
        const double d = fma(E, cp[p], 1.0);
        // hardware reciprocal and two Newton steps: one step leaves an
        // error of one sign (r <= 1/d) of order 2^-46, which would bias N(mu)
        // low by up to N_e 2^-46; after the second the error is rounding
        double r = __builtin_amdgcn_rcp(d);
        r = fma(r, fma(-d, r, 1.0), r);
        r = fma(r, fma(-d, r, 1.0), r);
        acc[p] = fma(ww, r, acc[p]);
      }
    });
  } else {
    for_terms(eps, w, nu_eff, M, nu, [&](double e, double ww) {
#pragma unroll
      for (int p = 0; p < MPTS; ++p) acc[p] = fma(ww, fermi_mu((e - s_pts[p]) / kT), acc[p]);
    });
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
    __shared__ double s_tmp[MTPB];
    const double tot = block_sum_partials(partials, (int)gridDim.x, 32, 0.0, OpAdd{}, s_tmp);
    if (tid < 32) s_N[tid] = tot;
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
  for_terms(eps, w, nu_eff, M, nu, [&](double e, double ww) {
    const double x = (e - mu) / kT;
    const double f = fermi_mu(x);
    v[0] = fma(ww * f, e, v[0]);
    v[1] = fma(ww, entropy_mu(x), v[1]);
    v[2] = fma(ww, f, v[2]);
  });
  reduce4(v);  // v[0] = total of value 2 b5 + b4
  if ((lane & 15) == 0) s_red[wv][((lane >> 5) & 1) * 2 + ((lane >> 4) & 1)] = v[0];
  __syncthreads();
  if (tid < 4) {
    double t = s_red[0][tid];
    for (int q = 1; q < MTPB / 64; ++q) t += s_red[q][tid];
    partials[4 * blockIdx.x + tid] = t;
  }
  if (last_block(st)) {
    __shared__ double s_tot[4];
    __shared__ double s_tmp[MTPB];
    const double tot = block_sum_partials(partials, (int)gridDim.x, 4, 0.0, OpAdd{}, s_tmp);
    if (tid < 4) s_tot[tid] = tot;
    __syncthreads();
    if (tid == 0) {
      st->E = s_tot[0];
      st->S_ent = s_tot[1];
      st->N = s_tot[2];
      st->counter = 0;
    }
  }
}

// state of a solve: the inputs of the bisection, everything else cleared
// (a kernel, so that a captured solve needs no host-to-device copy)
__global__ void mu_setup_kernel(MuState* st, double ne, double kT, double tol, double mu_fixed,
                                int fixed) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  MuState h{};
  h.ne = ne;
  h.kT = kT;
  h.tol = tol;
  if (fixed) {
    h.mu = mu_fixed;
    h.done = 1;
  }
  *st = h;
}

hipError_t launch_mu_setup(MuState* st, double ne, double kT, double tol, double mu_fixed,
                           int fixed, hipStream_t s) {
  hipLaunchKernelGGL(mu_setup_kernel, dim3(1), dim3(64), 0, s, st, ne, kT, tol, mu_fixed, fixed);
  return hipGetLastError();
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
