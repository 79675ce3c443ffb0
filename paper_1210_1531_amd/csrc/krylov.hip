// Per-column Krylov growth and projection (hot path of the multiple Arnoldi
// method: one Krylov subspace per column j of G = (zS - H)^-1, Eq. 1).
//
// One workgroup of 256 threads (4 waves) owns one column j = (J, alpha) at a
// time.  Its cluster C(J) is gathered in LDS as a local block-CSR over the
// global 4x4-block matrices (prologue), then nu Krylov steps run with the
// basis Q (n_C x nu) distributed over the registers of the workgroup: thread t
// owns cluster rows t, t + 256, t + 512.  Each step:
//   w = H_C q_k, z = S_C q_k       one fused SpMV (shared pattern and gathers)
//   h[:,k] = Q^T w, s[:,k] = Q^T z  projection, taken from the first
//                                   Gram-Schmidt pass's dot products
//   w -= Q h[:,k]; c = Q^T w; w -= Q c   classical Gram-Schmidt, twice
//   q_{k+1} = w / |w|                    (breakdown: |w| <= tol |H q_k|)
// The basis is Euclidean-orthonormal; it spans the same Krylov space
// K_nu(H_C; e_l) as the S-orthonormal basis of the method's reading, so the
// projected pencil (h, s) has the same Ritz pairs.  Dot products are reduced
// with a deterministic wave reduce-scatter plus a fixed-order cross-wave sum,
// so a column's result does not depend on which workgroup computes it.
#include "mag_internal.h"

namespace mag {

constexpr int KTPB = 256;
constexpr int KWAVES = KTPB / 64;
constexpr int ENT_MAX = CLUSTER_MAX * 28;  // local blocks of a cluster (average row <= 28)

// Sum NV = 2^LOG per-lane values over the wave.  Afterwards lane l holds the
// total of value index (l >> (6 - LOG)).  Deterministic for a fixed layout.
template <int LOG>
__device__ __forceinline__ double wave_reduce_scatter(double* v, int lane) {
#pragma unroll
  for (int step = 0; step < LOG; ++step) {
    const int off = 32 >> step;
    const bool up = (lane & off) != 0;
    constexpr int dummy = 0;
    (void)dummy;
    const int half = (1 << LOG) >> (step + 1);
#pragma unroll
    for (int t = 0; t < (1 << LOG) / 2; ++t) {
      if (t < half) {
        const double keep = up ? v[t + half] : v[t];
        const double send = up ? v[t] : v[t + half];
        v[t] = keep + __shfl_xor(send, off);
      }
    }
  }
  double x = v[0];
#pragma unroll
  for (int off = 32 >> LOG; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ __forceinline__ int lds_find(const int32_t* a, int n, int key) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = a[mid];
    if (v == key) return mid;
    if (v < key) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

template <int NU, int R>
__global__ __launch_bounds__(KTPB) void krylov_kernel(KrylovArgs a) {
  constexpr int NCH = (NU + 7) / 8;
  constexpr int RED = 16 * NCH + 8;
  __shared__ int32_t s_atoms[CLUSTER_MAX];
  __shared__ int32_t s_lptr[CLUSTER_MAX + 1];
  __shared__ int32_t s_lblk[ENT_MAX];
  __shared__ int16_t s_lcol[ENT_MAX];
  __shared__ int16_t s_pat[NC_MAX];
  __shared__ double s_x[NC_MAX];
  __shared__ double s_red[KWAVES][RED];
  __shared__ double s_fin[RED];
  __shared__ int s_misc[4];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cap = a.cap;

  for (int64_t it = 0;; ++it) {
    int64_t slot;
    if (a.queue) {
      if (tid == 0) s_misc[0] = atomicAdd(a.queue, 1);
      __syncthreads();
      slot = s_misc[0];
      __syncthreads();
    } else {
      if (it > 0) break;
      slot = blockIdx.x;
    }
    if (slot >= a.ncols) break;

    const int j = a.cols[slot];
    const int J = j >> 2;
    const int alpha = j & 3;
    const int64_t c0 = a.clus_ptr[J];
    const int nat = (int)(a.clus_ptr[J + 1] - c0);
    const int nC = NORB * nat;
    if (nat > CLUSTER_MAX || nC > KTPB * R || nat <= 0) {
      if (tid == 0) {
        atomicOr(a.err, (int)KERR_CAPACITY);
        a.nu_eff[slot] = 0;
      }
      continue;
    }

    // ---- prologue: cluster atoms and local block rows (gather of H_C, S_C)
    for (int i = tid; i < nat; i += KTPB) s_atoms[i] = a.clus_atoms[c0 + i];
    for (int i = tid; i < nC; i += KTPB) s_pat[i] = -1;
    __syncthreads();
    for (int i = tid; i < nat; i += KTPB) {
      const int I = s_atoms[i];
      int cnt = 0;
      for (int b = a.bptr[I]; b < a.bptr[I + 1]; ++b)
        if (lds_find(s_atoms, nat, a.bcol[b]) >= 0) ++cnt;
      s_lptr[i + 1] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
      int acc = 0;
      s_lptr[0] = 0;
      for (int i = 0; i < nat; ++i) {
        acc += s_lptr[i + 1];
        s_lptr[i + 1] = acc;
      }
      s_misc[1] = lds_find(s_atoms, nat, J);
    }
    __syncthreads();
    const int jl = s_misc[1];
    const int nent = s_lptr[nat];
    const int nbJ = a.bptr[J + 1] - a.bptr[J];
    const int nbJl = (jl >= 0) ? s_lptr[jl + 1] - s_lptr[jl] : -1;
    if (nent > ENT_MAX || jl < 0 || nbJl != nbJ) {
      if (tid == 0) {
        atomicOr(a.err, (int)(nent > ENT_MAX ? KERR_CAPACITY : KERR_PATTERN));
        a.nu_eff[slot] = 0;
      }
      __syncthreads();
      continue;
    }
    for (int i = tid; i < nat; i += KTPB) {
      const int I = s_atoms[i];
      int e = s_lptr[i];
      for (int b = a.bptr[I]; b < a.bptr[I + 1]; ++b) {
        const int kl = lds_find(s_atoms, nat, a.bcol[b]);
        if (kl >= 0) {
          s_lblk[e] = b;
          s_lcol[e] = (int16_t)kl;
          ++e;
        }
      }
    }
    __syncthreads();
    // pattern rows of column j: block row of J, in CSR order (block t, orbital)
    for (int t = tid; t < NORB * nbJ; t += KTPB) {
      const int kl = s_lcol[s_lptr[jl] + (t >> 2)];
      s_pat[NORB * kl + (t & 3)] = (int16_t)t;
    }
    const int ell = NORB * jl + alpha;
    for (int i = tid; i < nC; i += KTPB) s_x[i] = (i == ell) ? 1.0 : 0.0;

    double q[R][NU];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
#pragma unroll
      for (int i = 0; i < NU; ++i) q[rr][i] = 0.0;
      if (tid + KTPB * rr == ell) q[rr][0] = 1.0;
    }
    const int nu_max = min(a.nu, nC);
    int nu_eff = nu_max;
    double* hcol = a.hs + slot * (int64_t)(2 * cap * cap);
    double* scol = hcol + cap * cap;
    __syncthreads();

    for (int k = 0; k < nu_max; ++k) {
      // ---- fused SpMV: w = H_C q_k, z = S_C q_k
      double w[R], z[R];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int r = tid + KTPB * rr;
        double wa = 0.0, za = 0.0;
        if (r < nC) {
          const int il = r >> 2;
          const int ro = (r & 3) * 4;
          const int e1 = s_lptr[il + 1];
          for (int e = s_lptr[il]; e < e1; ++e) {
            const double* blk = a.bval + (int64_t)s_lblk[e] * 32 + ro;
            const double2 h01 = *reinterpret_cast<const double2*>(blk);
            const double2 h23 = *reinterpret_cast<const double2*>(blk + 2);
            const double2 s01 = *reinterpret_cast<const double2*>(blk + 16);
            const double2 s23 = *reinterpret_cast<const double2*>(blk + 18);
            const double* xv = s_x + NORB * s_lcol[e];
            const double2 x01 = *reinterpret_cast<const double2*>(xv);
            const double2 x23 = *reinterpret_cast<const double2*>(xv + 2);
            wa = fma(h01.x, x01.x, wa);
            wa = fma(h01.y, x01.y, wa);
            wa = fma(h23.x, x23.x, wa);
            wa = fma(h23.y, x23.y, wa);
            za = fma(s01.x, x01.x, za);
            za = fma(s01.y, x01.y, za);
            za = fma(s23.x, x23.x, za);
            za = fma(s23.y, x23.y, za);
          }
        }
        w[rr] = wa;
        z[rr] = za;
      }

      // ---- first Gram-Schmidt pass dot products = projection column k
      const int kc = k >> 3;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        if (c <= kc) {
          double v[16];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int i = c * 8 + t;
            double ph = 0.0, ps = 0.0;
            if (i < NU) {
#pragma unroll
              for (int rr = 0; rr < R; ++rr) {
                ph = fma(q[rr][i], w[rr], ph);
                ps = fma(q[rr][i], z[rr], ps);
              }
            }
            v[t] = ph;
            v[8 + t] = ps;
          }
          const double r = wave_reduce_scatter<4>(v, lane);
          if ((lane & 3) == 0) s_red[wave][c * 16 + (lane >> 2)] = r;
        }
      }
      {
        double ww = 0.0;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) ww = fma(w[rr], w[rr], ww);
        ww = wave_sum(ww);
        if (lane == 0) s_red[wave][16 * NCH] = ww;
      }
      __syncthreads();
      {
        const int nval = 16 * (kc + 1);
        for (int t = tid; t < nval; t += KTPB)
          s_fin[t] = ((s_red[0][t] + s_red[1][t]) + s_red[2][t]) + s_red[3][t];
        if (tid == 0)
          s_fin[16 * NCH] = ((s_red[0][16 * NCH] + s_red[1][16 * NCH]) + s_red[2][16 * NCH]) +
                            s_red[3][16 * NCH];
      }
      __syncthreads();
      const double ww1 = s_fin[16 * NCH];
      for (int i = tid; i <= k; i += KTPB) {
        hcol[(int64_t)k * cap + i] = s_fin[(i >> 3) * 16 + (i & 7)];
        scol[(int64_t)k * cap + i] = s_fin[(i >> 3) * 16 + 8 + (i & 7)];
      }
      if (!isfinite(ww1)) {
        if (tid == 0) atomicOr(a.err, (int)KERR_NONFINITE);
        nu_eff = k + 1;
        break;
      }
      if (k == nu_max - 1) break;

      // ---- w -= Q h[:, k]
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        if (c <= kc) {
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int i = c * 8 + t;
            if (i < NU) {
              const double hi = s_fin[c * 16 + t];
#pragma unroll
              for (int rr = 0; rr < R; ++rr) w[rr] = fma(-q[rr][i], hi, w[rr]);
            }
          }
        }
      }
      // ---- second pass: c = Q^T w
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        if (c <= kc) {
          double v[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int i = c * 8 + t;
            double p = 0.0;
            if (i < NU) {
#pragma unroll
              for (int rr = 0; rr < R; ++rr) p = fma(q[rr][i], w[rr], p);
            }
            v[t] = p;
          }
          const double r = wave_reduce_scatter<3>(v, lane);
          if ((lane & 7) == 0) s_red[wave][c * 8 + (lane >> 3)] = r;
        }
      }
      {
        double ww = 0.0;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) ww = fma(w[rr], w[rr], ww);
        ww = wave_sum(ww);
        if (lane == 0) s_red[wave][8 * NCH] = ww;
      }
      __syncthreads();
      {
        const int nval = 8 * (kc + 1);
        for (int t = tid; t < nval; t += KTPB)
          s_fin[t] = ((s_red[0][t] + s_red[1][t]) + s_red[2][t]) + s_red[3][t];
        if (tid == 0)
          s_fin[8 * NCH] = ((s_red[0][8 * NCH] + s_red[1][8 * NCH]) + s_red[2][8 * NCH]) +
                           s_red[3][8 * NCH];
      }
      __syncthreads();
      double csq = 0.0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        if (c <= kc) {
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int i = c * 8 + t;
            if (i < NU) {
              const double ci = s_fin[c * 8 + t];
              csq = fma(ci, ci, csq);
#pragma unroll
              for (int rr = 0; rr < R; ++rr) w[rr] = fma(-q[rr][i], ci, w[rr]);
            }
          }
        }
      }
      double beta2 = s_fin[8 * NCH] - csq;
      if (!(beta2 > 0.5 * s_fin[8 * NCH])) {
        // the second pass removed a large part: take the norm explicitly
        __syncthreads();
        double ww = 0.0;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) ww = fma(w[rr], w[rr], ww);
        ww = wave_sum(ww);
        if (lane == 0) s_red[wave][0] = ww;
        __syncthreads();
        beta2 = ((s_red[0][0] + s_red[1][0]) + s_red[2][0]) + s_red[3][0];
      }
      const double beta = sqrt(fmax(beta2, 0.0));
      if (!(beta > a.breakdown * sqrt(ww1))) {
        nu_eff = k + 1;
        break;
      }
      const double inv = 1.0 / beta;
#pragma unroll
      for (int rr = 0; rr < R; ++rr) w[rr] *= inv;
#pragma unroll
      for (int i = 1; i < NU; ++i) {
        if (i == k + 1) {
#pragma unroll
          for (int rr = 0; rr < R; ++rr) q[rr][i] = w[rr];
        }
      }
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int r = tid + KTPB * rr;
        if (r < nC) s_x[r] = w[rr];
      }
      __syncthreads();
    }

    // ---- epilogue: nu_eff, row l of Q, and the pattern (or all) rows of Q
    if (tid == 0) {
      a.nu_eff[slot] = nu_eff;
      if (a.npat) a.npat[slot] = a.full ? nC : NORB * nbJ;
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int r = tid + KTPB * rr;
      if (r < nC) {
        if (r == ell) {
          double* u = a.urow + slot * (int64_t)cap;
#pragma unroll
          for (int i = 0; i < NU; ++i) u[i] = q[rr][i];
          for (int i = NU; i < cap; ++i) u[i] = 0.0;
        }
        const int p = a.full ? r : (int)s_pat[r];
        if (p >= 0) {
          double* dst = a.qpat + (slot * (int64_t)a.pat_stride + p) * cap;
#pragma unroll
          for (int i = 0; i < NU; ++i) dst[i] = q[rr][i];
          for (int i = NU; i < cap; ++i) dst[i] = 0.0;
        }
      }
    }
    __syncthreads();
  }
}

int krylov_capacity(int nu) {
  static const int caps[] = {12, 20, 30, 40, 48};
  for (int c : caps)
    if (nu <= c) return c;
  return 0;
}

template <int NU, int R>
static hipError_t launch_one(const KrylovArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((krylov_kernel<NU, R>), dim3(grid), dim3(KTPB), 0, s, a);
  return hipGetLastError();
}

template <int NU>
static hipError_t launch_r(const KrylovArgs& a, int R, int grid, hipStream_t s) {
  switch (R) {
    case 1: return launch_one<NU, 1>(a, grid, s);
    case 2: return launch_one<NU, 2>(a, grid, s);
    case 3: return launch_one<NU, 3>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_krylov(const KrylovArgs& a, int cap, int rows_per_thread, int grid,
                         hipStream_t s) {
  switch (cap) {
    case 12: return launch_r<12>(a, rows_per_thread, grid, s);
    case 20: return launch_r<20>(a, rows_per_thread, grid, s);
    case 30: return launch_r<30>(a, rows_per_thread, grid, s);
    case 40: return launch_r<40>(a, rows_per_thread, grid, s);
    case 48: return launch_r<48>(a, rows_per_thread, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int krylov_threads() { return KTPB; }

}  // namespace mag
