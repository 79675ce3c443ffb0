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
//     block of the column's scratch (by columns, 1 / L_ii on the diagonal),
//     the dense reflector rows v_k the s block, all zero past n.
//  2. QL (one lane per column): the implicit QL method with Wilkinson-type
//     shifts on T (diagonal d, subdiagonal e) gives the eigenvalues, in the
//     steps of EISPACK's imtql1/imtql2 (Martin & Wilkinson).  The plane
//     rotations of every sweep are recorded instead of applied, each at a
//     fixed place (sweep, plane), so each lane carries only d and e.  The
//     lanes of a wave run their sweeps in lockstep trips, each rotation step
//     straight-line code under a lane predicate.
//  3. vectors (one wave per column): Z_T is rebuilt by replaying the recorded
//     rotations on Z = I (lane i holds row i of Z; every register index is a
//     compile-time constant; the rotations come through scalar loads, eight
//     planes at a time, with the identity in planes outside the sweep), then
//     c = L^-T Q_H Z_T column by column (lane k holds eigenvector k), so
//     h c = eps s c and c^T s c = I.  Then
//       d = c^T u = (Qc)^T e_l,  g = c^T s e_1 = (Qc)^T S_C e_l  (q_1 = e_l),
//       w_k = 2 d_k g_k (spin factor 2), eigenpairs ranked ascending,
//     and optionally P_pk = (Q_pat c)_pk d_k on the pattern rows, from which
//     pass 2 forms rho = 2 P f and pi = 2 P (f eps) (Eq. 2 on the Ritz
//     spectrum).
//  A column whose sweeps would overflow the record (or whose QL did not
//  converge in the lane kernel) is finished by a fallback kernel that runs
//  the same QL inside one wave with the rotations applied directly.
#include <algorithm>

#include "mag_internal.h"
#include "wave.h"

namespace mag {

constexpr int ETPB = 64;
constexpr int QL_MAXIT = 60;  // QL iterations per eigenvalue before giving up

// rotation records: sweep q, plane i at q * eig_sweep_stride + i (planes padded to a
// multiple of eight so that the replay loads whole groups of eight)
constexpr int eig_sweep_stride(int cap) { return (cap - 1 + 7) / 8 * 8; }
int eig_sweep_cap(int cap) { return std::min(4 * cap, 128); }
int eig_rec_cap(int cap) { return eig_sweep_cap(cap) * eig_sweep_stride(cap); }

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
  if (lane < NM) tr[3 * NM + lane] = L[0];  // s e_1 (zero past n)

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
  // L by columns over h (column t at t * NM), 1 / L_tt on the diagonal, zero
  // above it and past n
  if (lane < NM) {
#pragma unroll
    for (int t = 0; t < NM; ++t)
      h[t * NM + lane] = (row && t < n && t <= lane) ? ((t == lane) ? linv : L[t]) : 0.0;
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
      if (lane < NM) s[j * NM + lane] = vi;  // dense reflector row j (zero past n)
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
// 2. QL on the tridiagonal, one lane per column, rotations recorded per sweep.
// The lanes of a wave sit at different eigenvalues l and sweep lengths, so
// the loop is flattened into trips: in each trip a lane either deflates
// (ms == l: l advances) or runs one sweep.  Every rotation slot of a sweep is
// straight-line code under a lane predicate (values selected, not branched
// over), and a slot that no lane of the wave needs is skipped as a whole.
template <int NM>
__global__ __launch_bounds__(ETPB) void ql_kernel(EigArgs a) {
  const int64_t slot = (int64_t)blockIdx.x * ETPB + threadIdx.x;
  if (slot >= a.ncols) return;  // no barriers or cross-lane reads of dead lanes below
  const int n = a.nu_eff_in[slot];
  if (n <= 0 || n > NM) {
    a.qlst[slot] = 0;
    return;
  }
  const double* tr = a.trid + slot * (int64_t)(4 * NM);
  double d[NM], e[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) {  // whole rows (in bounds), entries past n replaced
    const double dt = tr[t], et = tr[NM + t];
    d[t] = (t < n) ? dt : 0.0;
    e[t] = (t < n) ? et : 0.0;
  }
  double2* rec = reinterpret_cast<double2*>(a.rot) + slot * (int64_t)a.rec_cap;
  int32_t* sw = a.sweep + slot * (int64_t)a.sweep_cap;
  constexpr int SWS = eig_sweep_stride(NM);
  int nsw = 0, status = 0, l = 0, iter = 0;
  for (;;) {
    const bool live = status == 0 && l < n;
    if (__builtin_amdgcn_ballot_w64(live) == 0) break;
    // ms: the first negligible subdiagonal at or after l.  e is zero from
    // n - 1 on, so ms = n - 1 when none is negligible before it
    int ms = NM - 1;
    double dm = d[NM - 1];
#pragma unroll
    for (int t = NM - 2; t >= 0; --t) {
      const bool neg = t >= l && fabs(e[t]) <= 0x1p-52 * (fabs(d[t]) + fabs(d[t + 1]));
      ms = neg ? t : ms;
      dm = neg ? d[t] : dm;
    }
    bool sweep = live && ms != l;
    if (live && ms == l) {
      ++l;
      iter = 0;
    }
    if (sweep && iter >= QL_MAXIT) {
      status = -2;
      sweep = false;
    }
    if (sweep && nsw >= a.sweep_cap) {
      status = -1;
      sweep = false;
    }
    if (__builtin_amdgcn_ballot_w64(sweep) == 0) continue;
    // Wilkinson-type shift from the leading 2 x 2 block at l
    double dl = 0.0, dl1 = 0.0, el = 1.0;
#pragma unroll
    for (int t = 0; t < NM; ++t) {
      dl = (t == l) ? d[t] : dl;
      el = (sweep && t == l) ? e[t] : el;
      dl1 = (t == l + 1) ? d[t] : dl1;
    }
    double g = (dl1 - dl) / (2.0 * el);
    double r = sqrt(fma(g, g, 1.0));
    g = dm - dl + el / (g + copysign(r, g));
    double sn = 1.0, cs = 1.0, p = 0.0;
    bool under = false;
    int cnt = 0;
    // slot i rotates the plane (i, i+1); the sweep runs i = ms-1 down to l.
    // Its last step (i = l, unless it ended early by underflow) also takes
    // d[l] -= p, e[l] = g, and its first step leaves e[ms] = 0
#pragma unroll
    for (int i = NM - 2; i >= 0; --i) {
      const bool act = sweep && i < ms && i >= l && !under;
      if (__builtin_amdgcn_ballot_w64(act) == 0) continue;
      const double f = sn * e[i], b = cs * e[i];
      // r = |(f, g)|; r == 0 only by underflow, and then the identity rotation
      // (sn, cs) = (0, 1) gives d[i+1] -= p, and the sweep ends
      const double q = fma(f, f, g * g);
      const bool bad = !(q > 0.0);
      const double rinv = bad ? 0.0 : rsqrt(bad ? 1.0 : q);
      const double sn1 = f * rinv;
      const double cs1 = bad ? 1.0 : g * rinv;
      const double g1 = d[i + 1] - p;
      const double r1 = fma(d[i] - g1, sn1, 2.0 * cs1 * b);
      const double p1 = sn1 * r1;
      const double g2 = fma(cs1, r1, -b);
      if (act) rec[nsw * SWS + i] = make_double2(sn1, cs1);
      e[i + 1] = act ? ((i + 1 == ms) ? 0.0 : q * rinv) : e[i + 1];
      d[i + 1] = act ? g1 + p1 : d[i + 1];
      const bool fin = act && i == l && !bad;
      d[i] = fin ? d[i] - p1 : d[i];
      e[i] = fin ? g2 : e[i];
      sn = act ? sn1 : sn;
      cs = act ? cs1 : cs;
      p = act ? p1 : p;
      g = act ? g2 : g;
      under = under || (act && bad);
      cnt += act ? 1 : 0;
    }
    if (sweep) {
      sw[nsw++] = (ms << 8) | cnt;
      ++iter;
    }
  }
  double* ev = a.evu + slot * (int64_t)NM;
#pragma unroll
  for (int t = 0; t < NM; ++t) ev[t] = d[t];  // zero past n
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
// 3. eigenvectors, spectral weights and pattern rows.  One wave per column,
// lane k carries eigenvector k.  What this kernel reads of the column and
// every lane needs (rotation record, reflectors, L) was written by earlier
// kernels, so it is read through the constant address space: scalar loads
// into SGPRs that feed the FMAs directly.  The pattern rows of Q, one per
// lane, come by vector loads.
typedef const __attribute__((address_space(4))) double kdouble;
typedef const __attribute__((address_space(4))) int32_t kint;

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
  double* T = sm;            // NM x LD: rows of Z, read back as columns
  double* ev = T + NM * LD;  // eigenvalues (unsorted)
  // L by columns (1 / L_ii on the diagonal), the reflector rows, the
  // tridiagonal's scratch: all zero past n
  kdouble* hL = (kdouble*)(a.hs + slot * (int64_t)(2 * NM * NM));
  kdouble* hV = hL + NM * NM;
  kdouble* tr = (kdouble*)(a.trid + slot * (int64_t)(4 * NM));

  // ---- Z_T: rows of the identity, rotated (lane i holds row i)
  double z[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) z[t] = (t == lane) ? 1.0 : 0.0;
  if (!FB) {
    const int nsw = a.qlst[slot];
    constexpr int SWS = eig_sweep_stride(NM);
    kdouble* rec = (kdouble*)(a.rot + slot * (int64_t)(2 * a.rec_cap));  // (sn, cs) pairs
    kint* sw = (kint*)(a.sweep + slot * (int64_t)a.sweep_cap);
    // sweep (ms, cnt) rotated the planes i = ms-1 down to ms-cnt, in that order;
    // its record is read eight planes at a time (two 64-byte scalar loads)
    int hdr_next = nsw > 0 ? sw[0] : 0;
    for (int q = 0; q < nsw; ++q) {
      const int hdr = hdr_next;
      if (q + 1 < nsw) hdr_next = sw[q + 1];  // in flight with the first group's loads
      const int ms = hdr >> 8;
      const int lo = ms - (hdr & 255);
      kdouble* rq = rec + 2 * (int64_t)q * SWS;
#pragma unroll
      for (int c = SWS / 8 - 1; c >= 0; --c) {
        if (8 * c < ms && 8 * c + 8 > lo) {
          double rr[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) rr[u] = rq[16 * c + u];
#pragma unroll
          for (int u = 7; u >= 0; --u) {
            const int i = 8 * c + u;
            if (i > NM - 2) continue;
            // planes outside the sweep take the identity rotation (a scalar
            // select): no per-lane predication
            const bool on = i < ms && i >= lo;
            const double sn = on ? rr[2 * u] : 0.0, cs = on ? rr[2 * u + 1] : 1.0;
            const double zf = z[i + 1];
            z[i + 1] = fma(sn, z[i], cs * zf);
            z[i] = fma(cs, z[i], -sn * zf);
          }
        }
      }
    }
    if (lane < n) ev[lane] = a.evu[slot * (int64_t)NM + lane];
  } else {
    if (!ql_wave<NM>(a.trid + slot * (int64_t)(4 * NM), n, z, ev, lane) && lane == 0)
      atomicOr(a.err, (int)KERR_NOCONV);
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
  // ---- column `lane` of Z_T (zero past n for lanes below n)
  double y[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) y[t] = (lane < NM) ? T[t * LD + lane] : 0.0;
  // ---- y = P_0 P_1 ... P_{n-3} y
  for (int k = n - 3; k >= 0; --k) {
    const double beta = tr[2 * NM + k];
    kdouble* vk = hV + k * NM;
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
  // ---- c = L^-T y (back substitution from the last row; column i of L)
#pragma unroll
  for (int i = NM - 1; i >= 0; --i) {
    kdouble* Li = hL + i * NM;
    double x = y[i];
#pragma unroll
    for (int p = i + 1; p < NM; ++p) x = fma(-Li[p], y[p], x);
    y[i] = x * Li[i];
  }
  // ---- d = c^T u, g = c^T s e_1, w = 2 d g
  kdouble* uu = (kdouble*)(a.urow + slot * (int64_t)NM);
  double dk = 0.0, gk = 0.0;
#pragma unroll
  for (int t = 0; t < NM; ++t) {
    dk = fma(uu[t], y[t], dk);
    gk = fma(tr[3 * NM + t], y[t], gk);
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

  // ---- P = (Q_pat c) diag(d): lanes over pattern rows.  c_k d_k goes to LDS
  // (transposed: entry t of vector k at k * LD + t) with the ranks; each lane
  // loads its own row of Q_pat (contiguous rows: coalesced vector loads) and
  // forms its row of P from broadcast reads of the staged vectors
  if (a.P) {
    double* Cd = T;                                  // NM x LD (the transposes are done)
    int* rk = reinterpret_cast<int*>(ev + NM);       // NM ranks
    __syncthreads();                                 // every lane has read T and ev
    if (lane < NM) {
#pragma unroll
      for (int t = 0; t < NM; ++t) Cd[lane * LD + t] = (lane < n) ? y[t] * dk : 0.0;
      rk[lane] = rank;
    }
    __syncthreads();
    const int np = a.npat[slot];
    const int64_t base = a.pmode ? a.rowptr[j] : slot * (int64_t)a.pat_stride;
    const double* qp = a.qpat + slot * (int64_t)a.pat_stride * NM;
    for (int p0 = 0; p0 < np; p0 += ETPB) {
      const int p = p0 + lane;
      const bool row = p < np;
      double q[NM];
      const double* qr = qp + (int64_t)(row ? p : 0) * NM;
#pragma unroll
      for (int t = 0; t < NM; t += 2) {
        if (t + 1 < NM) {
          const double2 v = *reinterpret_cast<const double2*>(qr + t);
          q[t] = v.x;
          q[t + 1] = v.y;
        } else {
          q[t] = qr[t];
        }
      }
      double* Pr = a.P + (base + (row ? p : 0)) * nuo;
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        if (k < nuo) {
          const double* ck = Cd + k * LD;
          double y0 = 0.0, y1 = 0.0;
#pragma unroll
          for (int t = 0; t < NM; t += 2) {
            y0 = fma(q[t], ck[t], y0);
            if (t + 1 < NM) y1 = fma(q[t + 1], ck[t + 1], y1);
          }
          if (row) Pr[rk[k]] = y0 + y1;
        }
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
  const size_t lds3 = (size_t)NM * (NM + 1) * sizeof(double) + NM * sizeof(double) + NM * sizeof(int);
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
