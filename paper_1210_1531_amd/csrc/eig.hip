// Projected eigensolve and spectral data of each column (batched, one wave
// per column).
//
// Input per column: the projected pencil (h, s) = (Q^T H_C Q, Q^T S_C Q) of
// size n = nu_eff (upper triangles, column k rows i <= k), the row u = Q^T e_l
// and the pattern rows of Q.  Steps:
//   s = L L^T (Cholesky), C = L^-1 h L^-T, C = V diag(eps) V^T by the cyclic
//   Jacobi method (round-robin parallel ordering, n/2 rotations per round),
//   c = L^-T V (so h c = eps s c and c^T s c = I), eigenpairs sorted
//   ascending;
//   d = c^T u = (Qc)^T e_l,  g = c^T s e_1 = (Qc)^T S_C e_l  (q_1 = e_l),
//   weights w_k = 2 d_k g_k (spin factor 2);
//   optionally P_pk = (Q_pat c)_pk d_k on the pattern rows, from which pass 2
//   forms rho = 2 P f and pi = 2 P (f eps) (Eq. 2 on the Ritz spectrum).
#include "mag_internal.h"

namespace mag {

constexpr int ETPB = 64;
constexpr int MAXP = NU_MAX / 2;  // rotations per round at most

__device__ __forceinline__ double wave_sum64(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ __forceinline__ void round_robin(int m, int r, int p, int& i, int& j) {
  // circle method: player m-1 fixed, players 0..m-2 rotate with the round
  if (p == 0) {
    i = m - 1;
    j = r;
  } else {
    const int mm = m - 1;  // r, p < mm, so one conditional subtraction wraps
    i = r + p;
    i -= (i >= mm) ? mm : 0;
    j = r - p + mm;
    j -= (j >= mm) ? mm : 0;
  }
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
}

__global__ __launch_bounds__(ETPB) void eig_kernel(EigArgs a) {
  extern __shared__ double sm[];
  const int64_t slot = blockIdx.x;
  if (slot >= a.ncols) return;
  const int lane = threadIdx.x;
  const int cap = a.cap;
  const int n = a.nu_eff_in[slot];
  const int j = a.cols[slot];
  const int nuo = a.nu;
  const int64_t oi = a.out_by_slot ? slot : (int64_t)j;  // output row

  if (n <= 0) {
    for (int k = lane; k < nuo; k += ETPB) {
      a.eps[oi * nuo + k] = 0.0;
      a.w[oi * nuo + k] = 0.0;
    }
    if (lane == 0) a.nu_eff_out[oi] = 0;
    return;
  }
  const int m = n + (n & 1);  // even size; an odd n gets one decoupled dummy index
  const int ld = m + 1;
  const int half = m / 2;
  double* A = sm;                 // m x ld
  double* V = A + m * ld;         // m x ld
  double* L = V + m * ld;         // m x ld
  double2* rot = reinterpret_cast<double2*>(L + m * ld);  // (c, s) per pair, MAXP
  double* ev = reinterpret_cast<double*>(rot + MAXP);      // eigenvalues (64)
  double* dv = ev + 64;           // d (64)
  double* gv = dv + 64;           // g (64)
  double* uu = gv + 64;           // row l of Q (64)
  double* s0 = uu + 64;           // first row of s (64)
  int2* pij = reinterpret_cast<int2*>(s0 + 64);  // (i, j) per pair, MAXP
  int* perm = reinterpret_cast<int*>(pij + MAXP); // perm[rank] = eigen index (64)
  int* flag = perm + 64;
  int2* btab = reinterpret_cast<int2*>(flag + 4);  // (p, q) of each 2x2 block

  const double* h = a.hs + slot * (int64_t)(2 * cap * cap);
  const double* s = h + cap * cap;

  for (int idx = lane; idx < m * m; idx += ETPB) {
    const int i = idx / m, k = idx - (idx / m) * m;
    double hv = 0.0, sv = 0.0;
    if (i < n && k < n) {
      const int lo = min(i, k), hi = max(i, k);
      hv = h[(int64_t)hi * cap + lo];
      sv = s[(int64_t)hi * cap + lo];
    } else if (i == k) {
      sv = 1.0;  // dummy index: identity overlap, zero h
    }
    A[i * ld + k] = hv;
    L[i * ld + k] = sv;
  }
  if (lane < 64) {
    uu[lane] = (lane < n) ? a.urow[slot * (int64_t)cap + lane] : 0.0;
    s0[lane] = (lane < n) ? s[(int64_t)lane * cap + 0] : 0.0;  // s_{0 i} = s_{i 0}
  }
  if (lane == 0) flag[0] = 0;
  __syncthreads();

  // ---- Cholesky s = L L^T (lower triangle of L, in place)
  for (int c = 0; c < m; ++c) {
    if (lane == 0) {
      double d = L[c * ld + c];
      for (int p = 0; p < c; ++p) d -= L[c * ld + p] * L[c * ld + p];
      if (!(d > 0.0)) {
        flag[0] = 1;
        d = 1.0;
      }
      L[c * ld + c] = sqrt(d);
    }
    __syncthreads();
    for (int i = c + 1 + lane; i < m; i += ETPB) {
      double x = L[i * ld + c];
      for (int p = 0; p < c; ++p) x -= L[i * ld + p] * L[c * ld + p];
      L[i * ld + c] = x / L[c * ld + c];
    }
    __syncthreads();
  }
  if (flag[0]) {
    if (lane == 0) atomicOr(a.err, (int)KERR_NOTPD);
  }

  // ---- X = L^-1 h (into V), then C = L^-1 X^T (into A)
  for (int col = lane; col < m; col += ETPB) {
    for (int i = 0; i < m; ++i) {
      double x = A[i * ld + col];
      for (int p = 0; p < i; ++p) x -= L[i * ld + p] * V[p * ld + col];
      V[i * ld + col] = x / L[i * ld + i];
    }
  }
  __syncthreads();
  for (int col = lane; col < m; col += ETPB) {
    for (int i = 0; i < m; ++i) {
      double x = V[col * ld + i];
      for (int p = 0; p < i; ++p) x -= L[i * ld + p] * A[p * ld + col];
      A[i * ld + col] = x / L[i * ld + i];
    }
  }
  __syncthreads();
  for (int idx = lane; idx < m * m; idx += ETPB) {
    const int i = idx / m, k = idx - (idx / m) * m;
    if (i < k) {
      const double v = 0.5 * (A[i * ld + k] + A[k * ld + i]);
      A[i * ld + k] = v;
      A[k * ld + i] = v;
    }
    V[i * ld + k] = (i == k) ? 1.0 : 0.0;
  }
  __syncthreads();

  // ---- cyclic Jacobi with round-robin pairs; each round applies A <- J^T A J
  // by 2x2 blocks: block (p, q) of rows {i_p, j_p} and columns {i_q, j_q}
  // becomes R_p^T B R_q, so every block is read and written by one lane.
  const int nblk = half * (half + 1) / 2;  // blocks with p <= q
  for (int b = lane; b < nblk; b += ETPB) {  // static block table (p, q)
    int p = 0, rem = b;
    while (rem >= half - p) {
      rem -= half - p;
      ++p;
    }
    btab[b] = make_int2(p, p + rem);
  }
  // V rows: lane l updates row (l mod rows_span) for pairs p = l / rows_span + k * groups
  const int span = m <= 32 ? 32 : 64;
  const int vrow = lane & (span - 1);
  const int vgrp = lane / span;          // 0 or 1
  const int groups = ETPB / span;        // 2 or 1
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, tot = 0.0;
    if (lane < m) {
      for (int i = 0; i < m; ++i) {
        const double v = A[i * ld + lane];
        tot += v * v;
        off += (i != lane) ? v * v : 0.0;
      }
    }
    off = wave_sum64(off);
    tot = wave_sum64(tot);
    if (!(off > 1e-30 * tot)) break;
    for (int r = 0; r < m - 1; ++r) {
      if (lane < half) {
        int i, jj;
        round_robin(m, r, lane, i, jj);
        const double aij = A[i * ld + jj];
        double c = 1.0, sn = 0.0;
        if (aij != 0.0) {
          const double tau = (A[jj * ld + jj] - A[i * ld + i]) / (2.0 * aij);
          double t;
          if (fabs(tau) > 1e150) t = 0.5 / tau;
          else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
        }
        rot[lane] = make_double2(c, sn);
        pij[lane] = make_int2(i, jj);
      }
      __syncthreads();
      for (int b = lane; b < nblk; b += ETPB) {
        const int2 pq = btab[b];
        const int2 P = pij[pq.x], Q = pij[pq.y];
        const double2 rp = rot[pq.x], rq = rot[pq.y];
        const double x00 = A[P.x * ld + Q.x], x01 = A[P.x * ld + Q.y];
        const double x10 = A[P.y * ld + Q.x], x11 = A[P.y * ld + Q.y];
        // rows: new row i = c row_i - s row_j, new row j = s row_i + c row_j
        const double y00 = rp.x * x00 - rp.y * x10, y01 = rp.x * x01 - rp.y * x11;
        const double y10 = rp.y * x00 + rp.x * x10, y11 = rp.y * x01 + rp.x * x11;
        // columns: new col i = c col_i - s col_j, new col j = s col_i + c col_j
        const double z00 = rq.x * y00 - rq.y * y01, z01 = rq.y * y00 + rq.x * y01;
        const double z10 = rq.x * y10 - rq.y * y11, z11 = rq.y * y10 + rq.x * y11;
        A[P.x * ld + Q.x] = z00;
        A[P.x * ld + Q.y] = z01;
        A[P.y * ld + Q.x] = z10;
        A[P.y * ld + Q.y] = z11;
        if (pq.x != pq.y) {
          A[Q.x * ld + P.x] = z00;
          A[Q.y * ld + P.x] = z01;
          A[Q.x * ld + P.y] = z10;
          A[Q.y * ld + P.y] = z11;
        }
      }
      // V <- V J
      if (vrow < m) {
        double* vr = V + vrow * ld;
        for (int p = vgrp; p < half; p += groups) {
          const int2 P = pij[p];
          const double2 rp = rot[p];
          const double x = vr[P.x], y = vr[P.y];
          vr[P.x] = rp.x * x - rp.y * y;
          vr[P.y] = rp.y * x + rp.x * y;
        }
      }
      __syncthreads();
    }
  }

  // ---- eigenvalues, ascending order (ties by index), c = L^-T V
  for (int k = lane; k < m; k += ETPB) ev[k] = A[k * ld + k];
  __syncthreads();
  for (int k = lane; k < n; k += ETPB) {
    int rank = 0;
    const double e = ev[k];
    for (int q2 = 0; q2 < n; ++q2) {
      const double f = ev[q2];
      rank += (f < e || (f == e && q2 < k)) ? 1 : 0;
    }
    perm[rank] = k;
  }
  // back substitution L^T c = V, column by column (into A)
  for (int col = lane; col < n; col += ETPB) {
    for (int i = m - 1; i >= 0; --i) {
      double x = V[i * ld + col];
      for (int p = i + 1; p < m; ++p) x -= L[p * ld + i] * A[p * ld + col];
      A[i * ld + col] = x / L[i * ld + i];
    }
  }
  __syncthreads();

  // ---- d = c^T u, g = c^T s e_1, w = 2 d g
  for (int k = lane; k < n; k += ETPB) {
    double d = 0.0, g = 0.0;
    for (int i = 0; i < n; ++i) {
      const double cik = A[i * ld + k];
      d = fma(uu[i], cik, d);
      g = fma(s0[i], cik, g);
    }
    dv[k] = d;
    gv[k] = g;
  }
  __syncthreads();
  for (int rk = lane; rk < nuo; rk += ETPB) {
    double e = 0.0, wk = 0.0;
    if (rk < n) {
      const int k = perm[rk];
      e = ev[k];
      wk = G_SPIN * dv[k] * gv[k];
      if (!isfinite(e) || !isfinite(wk)) atomicOr(a.err, (int)KERR_NONFINITE);
    }
    a.eps[oi * nuo + rk] = e;
    a.w[oi * nuo + rk] = wk;
  }
  if (lane == 0) a.nu_eff_out[oi] = n;

  // ---- P = (Q_pat c) diag(d), columns in ascending eigenvalue order
  if (a.P) {
    const int np = a.npat[slot];
    const int64_t base = a.pmode ? a.rowptr[j] : slot * (int64_t)a.pat_stride;
    const double* qp = a.qpat + slot * (int64_t)a.pat_stride * cap;
    for (int rk = lane; rk < nuo; rk += ETPB) {
      const int k = rk < n ? perm[rk] : 0;
      const double dk = rk < n ? dv[k] : 0.0;
      for (int p = 0; p < np; ++p) {
        const double* qrow = qp + (int64_t)p * cap;
        double y = 0.0;
        if (rk < n)
          for (int i = 0; i < n; ++i) y = fma(qrow[i], A[i * ld + k], y);
        a.P[(base + p) * nuo + rk] = y * dk;
      }
    }
  }
}

hipError_t launch_eig(const EigArgs& a, hipStream_t s) {
  if (a.ncols <= 0) return hipSuccess;
  const int m = a.nu + (a.nu & 1);
  const size_t lds = (size_t)3 * m * (m + 1) * sizeof(double) + MAXP * sizeof(double2) +
                     5 * 64 * sizeof(double) + MAXP * sizeof(int2) + (64 + 4) * sizeof(int) +
                     (MAXP * (MAXP + 1) / 2) * sizeof(int2);
  hipLaunchKernelGGL(eig_kernel, dim3((unsigned)a.ncols), dim3(ETPB), lds, s, a);
  return hipGetLastError();
}

// rho = 2 P f, pi = 2 P (f eps) on the pattern of each column (pass 2)
__device__ __forceinline__ double fermi_dev(double x) {
  if (x > 0.0) {
    const double e = exp(-x);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + exp(x));
}

__global__ __launch_bounds__(ETPB) void density_kernel(DensityArgs a) {
  __shared__ double f[NU_MAX];
  __shared__ double fe[NU_MAX];
  const int64_t slot = blockIdx.x;
  if (slot >= a.ncols) return;
  const int lane = threadIdx.x;
  const int j = a.cols[slot];
  const int n = a.nu_eff[j];
  const double mu = a.st->mu, kT = a.st->kT;
  for (int k = lane; k < NU_MAX; k += ETPB) {
    double fk = 0.0, ek = 0.0;
    if (k < n) {
      const double e = a.eps[(int64_t)j * a.nu + k];
      fk = fermi_dev((e - mu) / kT);
      ek = fk * e;
    }
    f[k] = fk;
    fe[k] = ek;
  }
  __syncthreads();
  const int64_t r0 = a.rowptr[j];
  const int np = (int)(a.rowptr[j + 1] - r0);
  const int64_t base = a.pmode ? r0 : slot * (int64_t)a.pat_stride;
  for (int p = lane; p < np; p += ETPB) {
    const double* row = a.P + (base + p) * a.nu;
    double r = 0.0, e = 0.0;
    for (int k = 0; k < n; ++k) {
      r = fma(row[k], f[k], r);
      e = fma(row[k], fe[k], e);
    }
    a.rho[r0 + p] = G_SPIN * r;
    if (a.pi) a.pi[r0 + p] = G_SPIN * e;
  }
}

hipError_t launch_density(const DensityArgs& a, hipStream_t s) {
  if (a.ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(density_kernel, dim3((unsigned)a.ncols), dim3(ETPB), 0, s, a);
  return hipGetLastError();
}

// full cluster columns of rho (rows = every orbital of the cluster)
__global__ __launch_bounds__(ETPB) void cluster_rho_kernel(const double* P, int pat_stride,
                                                           const int32_t* cols, int64_t ncols,
                                                           const int32_t* npat,
                                                           const int64_t* out_off,
                                                           const double* eps,
                                                           const int32_t* nu_eff, int nu,
                                                           const MuState* st, double* out) {
  __shared__ double f[NU_MAX];
  const int64_t slot = blockIdx.x;
  if (slot >= ncols) return;
  const int lane = threadIdx.x;
  const int n = nu_eff[slot];
  for (int k = lane; k < NU_MAX; k += ETPB)
    f[k] = (k < n) ? fermi_dev((eps[slot * (int64_t)nu + k] - st->mu) / st->kT) : 0.0;
  __syncthreads();
  const int np = npat[slot];
  const int64_t base = slot * (int64_t)pat_stride;
  for (int p = lane; p < np; p += ETPB) {
    const double* row = P + (base + p) * nu;
    double r = 0.0;
    for (int k = 0; k < n; ++k) r = fma(row[k], f[k], r);
    out[out_off[slot] + p] = G_SPIN * r;
  }
}

hipError_t launch_cluster_rho(const double* P, int pat_stride, const int32_t* cols, int64_t ncols,
                              const int32_t* npat, const int64_t* out_off, const double* eps,
                              const int32_t* nu_eff, int nu, const MuState* st, double* out,
                              hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(cluster_rho_kernel, dim3((unsigned)ncols), dim3(ETPB), 0, s, P, pat_stride,
                     cols, ncols, npat, out_off, eps, nu_eff, nu, st, out);
  return hipGetLastError();
}

// Galerkin Green's-function columns: G_cj(z) = sum_k P_ck / (z - eps_k)
__global__ __launch_bounds__(ETPB) void green_kernel(const double* P, int pat_stride,
                                                     const int32_t* cols, int64_t ncols,
                                                     const int32_t* npat, const int64_t* out_off,
                                                     const double* eps, const int32_t* nu_eff,
                                                     int nu, const double* z, int nz,
                                                     double* out) {
  const int64_t slot = blockIdx.x;
  if (slot >= ncols) return;
  const int lane = threadIdx.x;
  const int n = nu_eff[slot];
  const int np = npat[slot];
  const int64_t base = slot * (int64_t)pat_stride;
  const double* e = eps + slot * (int64_t)nu;
  for (int qz = 0; qz < nz; ++qz) {
    const double zr = z[2 * qz], zi = z[2 * qz + 1];
    for (int p = lane; p < np; p += ETPB) {
      const double* row = P + (base + p) * nu;
      double gr = 0.0, gi = 0.0;
      for (int k = 0; k < n; ++k) {
        // 1 / (z - e_k) = conj(z - e_k) / |z - e_k|^2
        const double dr = zr - e[k];
        const double inv = 1.0 / (dr * dr + zi * zi);
        gr = fma(row[k], dr * inv, gr);
        gi = fma(row[k], -zi * inv, gi);
      }
      const int64_t o = 2 * (out_off[slot] + (int64_t)qz * np + p);
      out[o] = gr;
      out[o + 1] = gi;
    }
  }
}

hipError_t launch_green(const double* P, int pat_stride, const int32_t* cols, int64_t ncols,
                        const int32_t* npat, const int64_t* out_off, const double* eps,
                        const int32_t* nu_eff, int nu, const double* z, int nz, double* out,
                        hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(green_kernel, dim3((unsigned)ncols), dim3(ETPB), 0, s, P, pat_stride, cols,
                     ncols, npat, out_off, eps, nu_eff, nu, z, nz, out);
  return hipGetLastError();
}

}  // namespace mag
