// Projected eigensolve and spectral data of each column.
//
// Input per column: the projected pencil (h, s) = (Q^T H_C Q, Q^T S_C Q) of
// size n = nu_eff (upper triangles, column k rows i <= k), the row u = Q^T e_l
// and the pattern rows of Q.  The generalized problem h c = eps s c is solved
// in three batched kernels:
//
//  1. reduction (one wave per column): s = L L^T (Cholesky),
//     C = L^-1 h L^-T, and the Householder tridiagonalization
//     C = Q_H T Q_H^T, Q_H = P_0 P_1 ... P_{n-3}, P_k = I - beta_k v_k v_k^T
//     (Golub & Van Loan's house vectors, v_k[k+1] = 1).  L overwrites the h
//     block of the column's scratch, the dense reflector rows v_k the s block.
//  2. QL (one lane per column): the implicit QL method with Wilkinson-type
//     shifts on T (diagonal d, subdiagonal e) gives the eigenvalues.  The
//     plane rotations of every sweep are recorded instead of applied, so each
//     lane carries only d and e.
//  3. vectors (one wave per column): Z_T is rebuilt by replaying the recorded
//     rotations on Z = I (lane i holds row i of Z; every register index is a
//     compile-time constant), then c = L^-T Q_H Z_T column by column (lane k
//     holds eigenvector k), so h c = eps s c and c^T s c = I.  Then
//       d = c^T u = (Qc)^T e_l,  g = c^T s e_1 = (Qc)^T S_C e_l  (q_1 = e_l),
//       w_k = 2 d_k g_k (spin factor 2), eigenpairs ranked ascending,
//     and optionally P_pk = (Q_pat c)_pk d_k on the pattern rows, from which
//     pass 2 forms rho = 2 P f and pi = 2 P (f eps) (Eq. 2 on the Ritz
//     spectrum).
//  A column whose rotation record would overflow its fixed slots (or whose
//  QL did not converge in the lane kernel) is finished by a fallback kernel
//  that runs the same QL inside one wave with the rotations applied directly.
#include <algorithm>

#include "mag_internal.h"
#include "wave.h"

namespace mag {

constexpr int ETPB = 64;
constexpr int QL_MAXIT = 60;  // QL iterations per eigenvalue before giving up

int eig_rec_cap(int cap) { return 2 * cap * cap; }
int eig_sweep_cap(int cap) { return std::min(4 * cap, 128); }  // two header registers per lane

// ---------------------------------------------------------------------------
// 1. Cholesky, C = L^-1 h L^-T, Householder tridiagonalization.  Lane i keeps
// row i of s (then of L) and row i of h (then column i of Y = L^-1 h and of C)
// in registers; every step below is unrolled over the capacity NM, so each
// register index is a compile-time constant, and the values one lane needs
// from another come by v_readlane (a constant lane index).

// value of lane `src` (compile-time) in every lane
__device__ __forceinline__ double bcast(double v, int src) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), src),
                          __builtin_amdgcn_readlane(__double2loint(v), src));
}

template <int NM>
__global__ __launch_bounds__(ETPB) void tri_kernel(EigArgs a) {
  extern __shared__ double sm[];  // NM x (NM + 1): transposes
  constexpr int LD = NM + 1;
  const int64_t slot = blockIdx.x;
  if (slot >= a.ncols) return;
  const int lane = threadIdx.x;
  const int n = a.nu_eff_in[slot];
  if (n <= 0 || n > NM) {
    if (n > NM && lane == 0) atomicOr(a.err, (int)KERR_CAPACITY);
    return;
  }
  double* h = a.hs + slot * (int64_t)(2 * NM * NM);
  double* s = h + NM * NM;
  double* tr = a.trid + slot * (int64_t)(4 * NM);
  const bool row = lane < n;

  // rows `lane` of s and h (upper triangles: element (i, k), i <= k, at k * NM + i)
  double L[NM], X[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) {
    const int lo = min(lane, t), hi = max(lane, t);
    const bool in = row && t < n;
    L[t] = in ? s[hi * NM + lo] : 0.0;
    X[t] = in ? h[hi * NM + lo] : 0.0;
  }
  if (row) tr[3 * NM + lane] = L[0];  // s e_1

  // ---- Cholesky s = L L^T, column c after column c: row c comes from lane c
  bool notpd = false;
  double linv = 0.0;  // 1 / L[lane][lane]
#pragma unroll
  for (int c = 0; c < NM; ++c) {
    if (c < n) {
      double acc = L[c];
#pragma unroll
      for (int p = 0; p < c; ++p) acc = fma(-L[p], bcast(L[p], c), acc);
      double d = bcast(acc, c);
      if (!(d > 0.0)) {
        notpd = true;
        d = 1.0;
      }
      const double r = sqrt(d), ri = 1.0 / r;
      if (lane == c) linv = ri;
      L[c] = (lane == c) ? r : ((lane > c) ? acc * ri : 0.0);
    }
  }
  if (notpd && lane == 0) atomicOr(a.err, (int)KERR_NOTPD);

  // ---- Y = L^-1 h: lane k solves for column k (row k of the symmetric h)
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    if (i < n) {
      double acc = X[i];
#pragma unroll
      for (int p = 0; p < i; ++p) acc = fma(-bcast(L[p], i), X[p], acc);
      X[i] = acc * bcast(linv, i);
    }
  }
  // row k of Y through LDS, then C = L^-1 Y^T column by column
  if (lane < NM) {
#pragma unroll
    for (int t = 0; t < NM; ++t) sm[t * LD + lane] = X[t];
  }
  __syncthreads();
  if (lane < NM) {
#pragma unroll
    for (int t = 0; t < NM; ++t) X[t] = sm[lane * LD + t];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    if (i < n) {
      double acc = X[i];
#pragma unroll
      for (int p = 0; p < i; ++p) acc = fma(-bcast(L[p], i), X[p], acc);
      X[i] = acc * bcast(linv, i);
    }
  }
  // symmetrize: C = (C + C^T) / 2, lane k keeping column k
  if (lane < NM) {
#pragma unroll
    for (int t = 0; t < NM; ++t) sm[t * LD + lane] = X[t];
  }
  __syncthreads();
  if (lane < NM) {
#pragma unroll
    for (int t = 0; t < NM; ++t) X[t] = 0.5 * (X[t] + sm[lane * LD + t]);
  }
  // L (zero above the diagonal) over h
  if (row) {
#pragma unroll
    for (int t = 0; t < NM; ++t)
      if (t < n) h[lane * NM + t] = (t <= lane) ? L[t] : 0.0;
  }

  // ---- Householder: step j reflects rows and columns j+1..n-1 so that column
  // j vanishes below the subdiagonal (Golub & Van Loan's house vector,
  // v[j+1] = 1).  Lane k keeps column k of the trailing block; C is symmetric,
  // so lane i's entry j is C[j][i] = C[i][j], its own part of column j.
#pragma unroll
  for (int j = 0; j + 2 < NM; ++j) {
    if (j + 2 < n) {
      const double x0 = bcast(X[j], j + 1);
      const double xi = (lane > j + 1 && row) ? X[j] : 0.0;
      const double sig = wave_allreduce(xi * xi);
      double beta = 0.0, v0 = 1.0, sub = x0;
      if (sig > 0.0) {
        const double mu = sqrt(x0 * x0 + sig);
        v0 = (x0 <= 0.0) ? x0 - mu : -sig / (x0 + mu);
        beta = 2.0 * v0 * v0 / (sig + v0 * v0);
        sub = mu;
      }
      const bool act = lane > j && row;                          // rows j+1..n-1
      const double vi = act ? ((lane == j + 1) ? 1.0 : xi / v0) : 0.0;
      if (lane == j) {
        tr[j] = X[j];
        tr[NM + j] = sub;
        tr[2 * NM + j] = beta;
      }
      if (row) s[j * NM + lane] = vi;  // dense reflector row j
      if (beta != 0.0) {
        // p = beta C v (lane k: its column against v), w = p - (beta p^T v / 2) v
        double vb[NM];
        double p = 0.0;
#pragma unroll
        for (int i = 0; i < NM; ++i) {
          vb[i] = 0.0;
          if (i > j && i < n) {
            vb[i] = bcast(vi, i);
            p = fma(X[i], vb[i], p);
          }
        }
        p = act ? beta * p : 0.0;
        const double kk = 0.5 * beta * wave_allreduce(p * vi);
        const double wi = p - kk * vi;
#pragma unroll
        for (int i = 0; i < NM; ++i) {
          if (i > j && i < n) {
            const double wb = bcast(wi, i);
            if (act) X[i] -= vb[i] * wi + wb * vi;
          }
        }
      }
    }
  }
  // the last 2 x 2 block (or 1 x 1)
#pragma unroll
  for (int t = 0; t < NM; ++t) {
    if (t + 2 == n) {
      const double dd = bcast(X[t], t), ee = bcast(X[t], t + 1);
      if (lane == 0) {
        tr[t] = dd;
        tr[NM + t] = ee;
        tr[2 * NM + t] = 0.0;
      }
    }
    if (t + 1 == n) {
      const double dd = bcast(X[t], t);
      if (lane == 0) {
        tr[t] = dd;
        tr[NM + t] = 0.0;
        tr[2 * NM + t] = 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 2. QL on the tridiagonal, one lane per column, rotations recorded per sweep
template <int NM>
__global__ __launch_bounds__(ETPB) void ql_kernel(EigArgs a) {
  const int64_t slot = (int64_t)blockIdx.x * ETPB + threadIdx.x;
  if (slot >= a.ncols) return;  // no barriers below
  const int n = a.nu_eff_in[slot];
  if (n <= 0 || n > NM) {
    a.qlst[slot] = 0;
    return;
  }
  const double* tr = a.trid + slot * (int64_t)(4 * NM);
  double d[NM], e[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) {
    d[t] = (t < n) ? tr[t] : 0.0;
    e[t] = (t < n) ? tr[NM + t] : 0.0;
  }
  double2* rec = reinterpret_cast<double2*>(a.rot) + slot * (int64_t)a.rec_cap;
  int32_t* sw = a.sweep + slot * (int64_t)a.sweep_cap;
  int nrec = 0, nsw = 0, status = 0;
  for (int l = 0; l < n && status == 0; ++l) {
    for (int iter = 0;; ++iter) {
      int ms = n - 1;
#pragma unroll
      for (int t = NM - 2; t >= 0; --t) {
        if (t >= l && t < n - 1) {
          if (fabs(e[t]) <= 0x1p-52 * (fabs(d[t]) + fabs(d[t + 1]))) ms = t;
        }
      }
      if (ms == l) break;
      if (iter >= QL_MAXIT) {
        status = -2;
        break;
      }
      if (nsw >= a.sweep_cap || nrec + (ms - l) > a.rec_cap) {
        status = -1;
        break;
      }
      double dl = 0.0, dl1 = 0.0, el = 0.0, dm = 0.0;
#pragma unroll
      for (int t = 0; t < NM; ++t) {
        if (t == l) {
          dl = d[t];
          el = e[t];
        }
        if (t == l + 1) dl1 = d[t];
        if (t == ms) dm = d[t];
      }
      double g = (dl1 - dl) / (2.0 * el);
      double r = sqrt(fma(g, g, 1.0));
      g = dm - dl + el / (g + copysign(r, g));
      double sn = 1.0, cs = 1.0, p = 0.0;
      bool under = false;
      int cnt = 0;
#pragma unroll
      for (int i = NM - 2; i >= 0; --i) {
        if (i >= ms) continue;
        if (i < l || under) break;
        const double f = sn * e[i], b = cs * e[i];
        // r = |(f, g)|; r == 0 only by underflow, and then the identity rotation
        // (sn, cs) = (0, 1) gives d[i+1] -= p, and the sweep ends
        const double q = fma(f, f, g * g);
        const bool bad = !(q > 0.0);
        const double rinv = bad ? 0.0 : rsqrt(q);
        r = q * rinv;
        e[i + 1] = r;
        sn = f * rinv;
        cs = bad ? 1.0 : g * rinv;
        g = d[i + 1] - p;
        r = fma(d[i] - g, sn, 2.0 * cs * b);
        p = sn * r;
        d[i + 1] = g + p;
        g = fma(cs, r, -b);
        rec[nrec + cnt] = make_double2(sn, cs);
        ++cnt;
        under = bad;
      }
      sw[nsw++] = (ms << 8) | cnt;
      nrec += cnt;
#pragma unroll
      for (int t = 0; t < NM; ++t) {
        if (!under && t == l) {
          d[t] -= p;
          e[t] = g;
        }
        if (t == ms) e[t] = 0.0;
      }
    }
  }
  double* ev = a.evu + slot * (int64_t)NM;
#pragma unroll
  for (int t = 0; t < NM; ++t)
    if (t < n) ev[t] = d[t];
  a.qlst[slot] = (status == 0) ? nsw : status;
  if (status != 0) a.fb_list[atomicAdd(a.fb_count, 1)] = (int32_t)slot;
}

// the same QL inside one wave, rotations applied to the row of Z held by each lane
template <int NM>
__device__ __forceinline__ bool ql_wave(const double* tr, int n, double* z, double* ev, int lane) {
  double d[NM], e[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) {
    d[t] = (t < n) ? tr[t] : 0.0;
    e[t] = (t < n) ? tr[NM + t] : 0.0;
  }
  bool ok = true;
  for (int l = 0; l < n && ok; ++l) {
    for (int iter = 0;; ++iter) {
      int ms = n - 1;
#pragma unroll
      for (int t = NM - 2; t >= 0; --t) {
        if (t >= l && t < n - 1) {
          if (fabs(e[t]) <= 0x1p-52 * (fabs(d[t]) + fabs(d[t + 1]))) ms = t;
        }
      }
      ms = __builtin_amdgcn_readfirstlane(ms);
      if (ms == l) break;
      if (iter >= QL_MAXIT) {
        ok = false;
        break;
      }
      double dl = 0.0, dl1 = 0.0, el = 0.0, dm = 0.0;
#pragma unroll
      for (int t = 0; t < NM; ++t) {
        if (t == l) {
          dl = d[t];
          el = e[t];
        }
        if (t == l + 1) dl1 = d[t];
        if (t == ms) dm = d[t];
      }
      double g = (dl1 - dl) / (2.0 * el);
      double r = sqrt(fma(g, g, 1.0));
      g = dm - dl + el / (g + copysign(r, g));
      double sn = 1.0, cs = 1.0, p = 0.0;
      bool under = false;
#pragma unroll
      for (int i = NM - 2; i >= 0; --i) {
        if (i >= ms) continue;
        if (i < l || under) break;
        const double f = sn * e[i], b = cs * e[i];
        const double q = fma(f, f, g * g);
        const bool bad = !(q > 0.0);
        const double rinv = bad ? 0.0 : rsqrt(q);
        r = q * rinv;
        e[i + 1] = r;
        sn = f * rinv;
        cs = bad ? 1.0 : g * rinv;
        g = d[i + 1] - p;
        r = fma(d[i] - g, sn, 2.0 * cs * b);
        p = sn * r;
        d[i + 1] = g + p;
        g = fma(cs, r, -b);
        const double zf = z[i + 1];
        z[i + 1] = fma(sn, z[i], cs * zf);
        z[i] = fma(cs, z[i], -sn * zf);
        under = __builtin_amdgcn_readfirstlane((int)bad) != 0;
      }
#pragma unroll
      for (int t = 0; t < NM; ++t) {
        if (!under && t == l) {
          d[t] -= p;
          e[t] = g;
        }
        if (t == ms) e[t] = 0.0;
      }
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < NM; ++t)
      if (t < n) ev[t] = d[t];
  }
  return ok;
}

// ---------------------------------------------------------------------------
// 3. eigenvectors, spectral weights and pattern rows
template <int NM, bool FB>
__device__ __forceinline__ void vectors_column(const EigArgs& a, int64_t slot, double* sm) {
  constexpr int LD = NM + 1;
  const int lane = threadIdx.x;
  const int n = a.nu_eff_in[slot];
  const int j = a.cols[slot];
  const int nuo = a.nu;
  const int64_t oi = a.out_by_slot ? slot : (int64_t)j;  // output row
  if (n <= 0 || n > NM) {
    for (int k = lane; k < nuo; k += ETPB) {
      a.eps[oi * nuo + k] = 0.0;
      a.w[oi * nuo + k] = 0.0;
    }
    if (lane == 0) a.nu_eff_out[oi] = 0;
    return;
  }
  double* T = sm;              // NM x LD: rows of Z, then the reflectors
  double* Lm = T + NM * LD;    // NM x LD: L, zero padded
  double* uu = Lm + NM * LD;   // row l of Q
  double* s0 = uu + NM;        // s e_1
  double* li = s0 + NM;        // 1 / L_ii
  double* ev = li + NM;        // eigenvalues (unsorted)
  const double* hL = a.hs + slot * (int64_t)(2 * NM * NM);
  const double* hV = hL + NM * NM;
  const double* tr = a.trid + slot * (int64_t)(4 * NM);

  for (int idx = lane; idx < NM * NM; idx += ETPB) {
    const int i = idx / NM, k = idx - (idx / NM) * NM;
    Lm[i * LD + k] = (i < n && k < n) ? hL[i * NM + k] : 0.0;
  }
  if (lane < NM) {
    uu[lane] = (lane < n) ? a.urow[slot * (int64_t)NM + lane] : 0.0;
    s0[lane] = (lane < n) ? tr[3 * NM + lane] : 0.0;
    li[lane] = (lane < n) ? 1.0 / hL[lane * NM + lane] : 0.0;
  }

  // ---- Z_T: rows of the identity, rotated
  double z[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) z[t] = (t == lane) ? 1.0 : 0.0;
  if (!FB) {
    const int nsw = a.qlst[slot];
    const double2* rec = reinterpret_cast<const double2*>(a.rot) + slot * (int64_t)a.rec_cap;
    const int32_t* sw = a.sweep + slot * (int64_t)a.sweep_cap;
    // every sweep header in registers (lane q holds sweeps q and q + 64), and
    // the next sweep's rotations loaded while the current one is applied
    const int h0 = lane < nsw ? sw[lane] : 0;
    const int h1 = lane + 64 < nsw ? sw[lane + 64] : 0;
    auto header = [&](int q) {
      return q < 64 ? __builtin_amdgcn_readlane(h0, q) : __builtin_amdgcn_readlane(h1, q - 64);
    };
    // lane t holds the rotation of the plane (t, t+1); sweep (ms, cnt) ran t = ms-1 down to ms-cnt
    auto fetch = [&](int hdr, int ptr) {
      const int ms = hdr >> 8, lo = ms - (hdr & 255);
      double2 r = make_double2(0.0, 1.0);
      if (lane < ms && lane >= lo) r = rec[ptr + (ms - 1 - lane)];
      return r;
    };
    int hdr = nsw > 0 ? header(0) : 0;
    int ptr = 0;
    double2 next = fetch(hdr, 0);
    for (int q = 0; q < nsw; ++q) {
      const int ms = hdr >> 8, cnt = hdr & 255;
      const int lo = ms - cnt;
      const double2 rt = next;
      const int ptr_n = ptr + cnt;
      const int hdr_n = (q + 1 < nsw) ? header(q + 1) : 0;
      if (q + 1 < nsw) next = fetch(hdr_n, ptr_n);
#pragma unroll
      for (int i = NM - 2; i >= 0; --i) {
        if (i < ms && i >= lo) {
          const double sn = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(rt.x), i),
                                             __builtin_amdgcn_readlane(__double2loint(rt.x), i));
          const double cs = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(rt.y), i),
                                             __builtin_amdgcn_readlane(__double2loint(rt.y), i));
          const double zf = z[i + 1];
          z[i + 1] = fma(sn, z[i], cs * zf);
          z[i] = fma(cs, z[i], -sn * zf);
        }
      }
      hdr = hdr_n;
      ptr = ptr_n;
    }
    if (lane < n) ev[lane] = a.evu[slot * (int64_t)NM + lane];
  } else {
    if (!ql_wave<NM>(tr, n, z, ev, lane) && lane == 0) atomicOr(a.err, (int)KERR_NOCONV);
  }
  if (lane < NM) {
#pragma unroll
    for (int t = 0; t < NM; ++t) T[lane * LD + t] = z[t];
  }
  __syncthreads();
  // ---- rank of eigenvalue `lane` (ascending, ties by index)
  int rank = lane;
  double ek = 0.0;
  if (lane < n) {
    ek = ev[lane];
    rank = 0;
    for (int q2 = 0; q2 < n; ++q2) {
      const double f = ev[q2];
      rank += (f < ek || (f == ek && q2 < lane)) ? 1 : 0;
    }
  }
  // ---- column `lane` of Z_T
  double y[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) y[t] = (lane < NM) ? T[t * LD + lane] : 0.0;
  __syncthreads();
  for (int idx = lane; idx < NM * NM; idx += ETPB) {
    const int k = idx / NM, i = idx - (idx / NM) * NM;
    T[k * LD + i] = (k + 2 < n && i < n) ? hV[k * NM + i] : 0.0;
  }
  __syncthreads();
  // ---- y = P_0 P_1 ... P_{n-3} y
  for (int k = n - 3; k >= 0; --k) {
    const double beta = tr[2 * NM + k];
    const double* vk = T + k * LD;
    double r0 = 0.0, r1 = 0.0;
#pragma unroll
    for (int t = 0; t < NM; t += 2) {
      r0 = fma(vk[t], y[t], r0);
      if (t + 1 < NM) r1 = fma(vk[t + 1], y[t + 1], r1);
    }
    const double r = beta * (r0 + r1);
#pragma unroll
    for (int t = 0; t < NM; ++t) y[t] = fma(-r, vk[t], y[t]);
  }
  // ---- c = L^-T y (back substitution from the last row)
#pragma unroll
  for (int i = NM - 1; i >= 0; --i) {
    double x = y[i];
#pragma unroll
    for (int p = i + 1; p < NM; ++p) x = fma(-Lm[p * LD + i], y[p], x);
    y[i] = x * li[i];
    __builtin_amdgcn_sched_barrier(0);  // bound the loads in flight to one row
  }
  // ---- d = c^T u, g = c^T s e_1, w = 2 d g
  double dk = 0.0, gk = 0.0;
#pragma unroll
  for (int t = 0; t < NM; ++t) {
    dk = fma(uu[t], y[t], dk);
    gk = fma(s0[t], y[t], gk);
  }
  const double wk = G_SPIN * dk * gk;
  if (a.cvec && lane < NM) {
    double* cv = a.cvec + slot * (int64_t)(NM * NM) + lane * NM;
#pragma unroll
    for (int t = 0; t < NM; ++t) cv[t] = (lane < n && t < n) ? y[t] : 0.0;
    double* cd = a.cdg + slot * (int64_t)(3 * NM);
    cd[lane] = (lane < n) ? ek : 0.0;
    cd[NM + lane] = (lane < n) ? dk : 0.0;
    cd[2 * NM + lane] = (lane < n) ? gk : 0.0;
  }
  if (lane < n) {
    if (!isfinite(ek) || !isfinite(wk)) atomicOr(a.err, (int)KERR_NONFINITE);
    a.eps[oi * nuo + rank] = ek;
    a.w[oi * nuo + rank] = wk;
  } else if (lane < nuo) {
    a.eps[oi * nuo + lane] = 0.0;
    a.w[oi * nuo + lane] = 0.0;
  }
  if (lane == 0) a.nu_eff_out[oi] = n;

  // ---- P = (Q_pat c) diag(d): row p, column rank(k)
  if (a.P) {
    const int np = a.npat[slot];
    const int64_t base = a.pmode ? a.rowptr[j] : slot * (int64_t)a.pat_stride;
    const double* qp = a.qpat + slot * (int64_t)a.pat_stride * NM;
    // the pattern rows of Q are staged in LDS (over Z and L, free now) in
    // chunks, with one coalesced copy per chunk, and read back as broadcasts
    constexpr int PCH = (2 * NM * LD) / NM;
    double* qs = T;
    for (int p0 = 0; p0 < np; p0 += PCH) {
      const int pc = min(PCH, np - p0);
      __syncthreads();
      for (int idx = lane; idx < pc * NM; idx += ETPB) qs[idx] = qp[(int64_t)p0 * NM + idx];
      __syncthreads();
      for (int p = 0; p < pc; ++p) {
        const double* qrow = qs + p * NM;
        double y0 = 0.0, y1 = 0.0;
#pragma unroll
        for (int t = 0; t < NM; t += 2) {
          y0 = fma(qrow[t], y[t], y0);
          if (t + 1 < NM) y1 = fma(qrow[t + 1], y[t + 1], y1);
        }
        if (lane < nuo) a.P[(base + p0 + p) * nuo + rank] = (lane < n) ? (y0 + y1) * dk : 0.0;
      }
    }
  }
}

template <int NM>
__global__ __launch_bounds__(ETPB) void vec_kernel(EigArgs a) {
  extern __shared__ double sm[];
  const int64_t slot = blockIdx.x;
  if (slot >= a.ncols) return;
  const int n = a.nu_eff_in[slot];
  if (n > 0 && n <= NM && a.qlst[slot] < 0) return;  // left to the fallback kernel
  vectors_column<NM, false>(a, slot, sm);
}

template <int NM>
__global__ __launch_bounds__(ETPB) void vec_fallback_kernel(EigArgs a) {
  extern __shared__ double sm[];
  const int cnt = *a.fb_count;
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) {
    vectors_column<NM, true>(a, a.fb_list[q], sm);
    __syncthreads();
  }
}

template <int NM>
static hipError_t launch_eig_nm(const EigArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)a.ncols;
  const size_t lds1 = (size_t)NM * (NM + 1) * sizeof(double);
  const size_t lds3 = (size_t)2 * NM * (NM + 1) * sizeof(double) + 4 * NM * sizeof(double);
  hipLaunchKernelGGL(tri_kernel<NM>, dim3(nb), dim3(ETPB), lds1, s, a);
  hipError_t e = launch_fill_i32(a.fb_count, 1, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ql_kernel<NM>, dim3((nb + ETPB - 1) / ETPB), dim3(ETPB), 0, s, a);
  hipLaunchKernelGGL(vec_kernel<NM>, dim3(nb), dim3(ETPB), lds3, s, a);
  hipLaunchKernelGGL(vec_fallback_kernel<NM>, dim3(std::min(nb, 256u)), dim3(ETPB), lds3, s, a);
  return hipGetLastError();
}

hipError_t launch_eig(const EigArgs& a, hipStream_t s) {
  if (a.ncols <= 0) return hipSuccess;
  switch (a.cap) {
    case 12: return launch_eig_nm<12>(a, s);
    case 20: return launch_eig_nm<20>(a, s);
    case 30: return launch_eig_nm<30>(a, s);
    case 40: return launch_eig_nm<40>(a, s);
    case 48: return launch_eig_nm<48>(a, s);
    default: return hipErrorInvalidValue;
  }
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

// energy-resolved crystal orbital Hamiltonian population (Eq. 4) per block of
// the pattern, broadened by eta: block t of block row J (column atom K),
//   C(e) = g_s sum_a sum_k c_ak L(e - eps_{j,k}),  j = 4J + a,
//   c_ak = sum_b H_{Ja;Kb} P_{Kb,j,k}  (P = Y d on the pattern of column j),
//   L(x) = (eta / pi) / (x^2 + eta^2)  = -Im 1/(x + i eta) / pi,
// from the stored pattern rows (P[(rowptr[j] + p) nu + k]) and the Ritz values
// of the last solve.  One workgroup per block: the 4 nu weights first, then
// lanes over the energies.
__global__ __launch_bounds__(ETPB) void cohp_kernel(const double* bval, const int32_t* bptr,
                                                    int64_t n, int64_t nblk,
                                                    const int64_t* rowptr, const double* P,
                                                    const double* eps, const int32_t* nu_eff,
                                                    int nu, const double* en, int ne, double eta,
                                                    double* out) {
  __shared__ double c_s[4 * 48], e_s[4 * 48];
  const int64_t b = blockIdx.x;
  if (b >= nblk) return;
  const int lane = threadIdx.x;
  int64_t lo = 0, hi = n - 1;  // block row J: last row with bptr[J] <= b
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (bptr[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const int64_t J = lo;
  const int t = (int)(b - bptr[J]);
  const double* hv = bval + b * 32;  // H: quarters of row pairs
  for (int idx = lane; idx < 4 * nu; idx += ETPB) {
    const int a = idx / nu, k = idx - (idx / nu) * nu;
    const int64_t j = 4 * J + a;
    double c = 0.0, e = 0.0;
    if (k < nu_eff[j]) {
      const double* pr = P + (rowptr[j] + 4 * t) * nu + k;
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) c = fma(hv[(c4 >> 1) * 8 + 2 * a + (c4 & 1)], pr[c4 * nu], c);
      e = eps[j * nu + k];
    }
    c_s[idx] = c;
    e_s[idx] = e;
  }
  __syncthreads();
  const double scale = G_SPIN * eta / 3.14159265358979323846;
  const double eta2 = eta * eta;
  for (int q = lane; q < ne; q += ETPB) {
    const double x = en[q];
    double acc = 0.0;
    for (int idx = 0; idx < 4 * nu; ++idx) {
      const double d = x - e_s[idx];
      // d^2 + eta^2 is a normal positive number (eta >= 1e-100 is checked
      // on entry): the hardware reciprocal and two Newton steps give it to
      // full precision with nothing to special-case
      const double den = fma(d, d, eta2);
      double r = __builtin_amdgcn_rcp(den);
      r = fma(r, fma(-den, r, 1.0), r);
      r = fma(r, fma(-den, r, 1.0), r);
      acc = fma(c_s[idx], r, acc);
    }
    out[b * ne + q] = scale * acc;
  }
}

hipError_t launch_cohp(const double* bval, const int32_t* bptr, int64_t n, int64_t nblk,
                       const int64_t* rowptr, const double* P, const double* eps,
                       const int32_t* nu_eff, int nu, const double* en, int ne, double eta,
                       double* out, hipStream_t s) {
  if (nblk <= 0 || ne <= 0) return hipSuccess;
  if (nu > 48) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cohp_kernel, dim3((unsigned)nblk), dim3(ETPB), 0, s, bval, bptr, n, nblk,
                     rowptr, P, eps, nu_eff, nu, en, ne, eta, out);
  return hipGetLastError();
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
