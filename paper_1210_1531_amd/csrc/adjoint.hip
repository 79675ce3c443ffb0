// Exact gradient of the truncated-Krylov grand potential with respect to the
// atomic positions (reverse mode through the Krylov construction).
//
// The method takes energies and forces through the density matrix (the force
// paragraph after Eq. 1, Eq. 2).  The forces through rho and pi are the
// derivative of the free energy only when every column's Krylov space is
// exact; with nu below the cluster dimension each column's Ritz data depend
// on H_C also through the space K_nu(H_C; e_l) itself.  Here the grand
// potential of column j,
//   Omega_j = sum_k w_k omega(eps_k),  omega(e) = -kT ln(1 + e^{-(e - mu)/kT}),
// is differentiated exactly, at fixed mu (the free energy at fixed electron
// number has the same position gradient), in three stages per column:
//
//  1. projected pencil: with c the Ritz vectors (h c = eps s c, c^T s c = I),
//     d = c^T e_1, g = c^T s e_1 and the divided differences
//     D_ab = (omega(eps_a) - omega(eps_b)) / (eps_a - eps_b) (omega' = f on
//     the diagonal), K_ab = D_ab d_a g_b gives (Daleckii-Krein)
//       hbar = c (K + K^T) c^T,   sbar = -c (K Lambda + Lambda K^T) c^T
//     (adj_prep_kernel);
//  2. the forward pass leaves each column's basis Q, its h, the beta_k and the
//     last step's residual in scratch; they are loaded back into registers
//     (the basis as the forward holds it), and the recurrence
//     q_{k+1} = (H q_k - Q_k t_k) / beta_k is run backwards.  The adjoint of every step needs only the next basis
//     vector's adjoint qbar_{k+1}:
//       rbar_k = (1 - q_{k+1} q_{k+1}^T) qbar_{k+1} / beta_k,
//       wbar_k = (1 - Q_{k+1} Q_{k+1}^T) qbar_{k+1} / beta_k,  Hbar += wbar_k q_k^T,
//     and qbar_{k+1} itself is assembled from the projection (2 H Q hbar +
//     2 S Q sbar, with H Q = Q h + r_nu e_nu^T), the step's own H wbar_{k+1},
//     the two-term band of t (alpha_{k+1} rbar_{k+1}, beta_{k+1} rbar_{k+2};
//     h is tridiagonal in exact arithmetic) and Q y_{k+1}, a combination of
//     the basis whose coefficients collect c_m = Q_m^T rbar_m through h.  One
//     fused SpMV (H wbar, S Q sbar e_i) and one set of dot products per step;
//  3. Hbar = Z Q^T (Z = Wbar + Q hbar) and Sbar = Q sbar Q^T are contracted,
//     block by block of the cluster, with the Slater-Koster derivatives:
//     for the pair (A, B), d = R_B - R_A,
//       G_AB = <dH_AB/dd, Z_A Q_B^T + Q_A Z_B^T> + <dS_AB/dd, 2 (Q sbar)_A Q_B^T>,
//     and atom A's force from column j is sum_B G_AB.  The basis and Z are
//     staged through LDS a few columns at a time.
//
// One workgroup owns one atom at a time and runs its four columns; the
// atom's force parts on its cluster atoms (fJ, indexed like the cluster
// list) are summed over the columns in LDS, and gather_forces_kernel adds,
// for every atom I, the parts that the clusters holding I computed for it
// (deterministic order).  A column whose Krylov space breaks down is
// differentiated at its dimension nu_eff.
#include <algorithm>

#include "mag_internal.h"
#include "sk_dev.h"
#include "wave.h"

namespace mag {

constexpr int AENT_MAX = CLUSTER_MAX * 24;

template <int KTPB>
__device__ __forceinline__ int adj_excl_scan(int v, int32_t* s_scan, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  if (lane == 63) s_scan[wave] = inc;
  __syncthreads();
  int base = 0, all = 0;
#pragma unroll
  for (int w = 0; w < KTPB / 64; ++w) {
    const int t = s_scan[w];
    if (w < wave) base += t;
    all += t;
  }
  __syncthreads();
  *total = all;
  return base + inc - v;
}

__device__ __forceinline__ int adj_find(const int32_t* a, int n, int key) {
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

// one row of the fused SpMV: hx = (H_C x)_r and, if S_TOO, sy = (S_C y)_r,
// over the row's local block entries [e0, e1); rp points at the row's values
// inside its global block row
template <bool S_TOO>
__device__ __forceinline__ void row_spmv(const double* rp, const uint16_t* s_ent, int e0, int e1,
                                         const double* x, const double* y, double& hx,
                                         double& sy) {
  double wa = 0.0, wb = 0.0, za = 0.0, zb = 0.0;
  int e = e0;
  for (; e + 1 < e1; e += 2) {
    const unsigned p0 = s_ent[e], p1 = s_ent[e + 1];
    const double* b0 = rp + (p0 >> 8) * 32;
    const double* b1 = rp + (p1 >> 8) * 32;
    const double2 h01 = *reinterpret_cast<const double2*>(b0);
    const double2 h23 = *reinterpret_cast<const double2*>(b0 + 8);
    const double2 g01 = *reinterpret_cast<const double2*>(b1);
    const double2 g23 = *reinterpret_cast<const double2*>(b1 + 8);
    const int k0 = NORB * (int)(p0 & 255), k1 = NORB * (int)(p1 & 255);
    const double2 x01 = *reinterpret_cast<const double2*>(x + k0);
    const double2 x23 = *reinterpret_cast<const double2*>(x + k0 + 2);
    const double2 u01 = *reinterpret_cast<const double2*>(x + k1);
    const double2 u23 = *reinterpret_cast<const double2*>(x + k1 + 2);
    wa = fma(h01.x, x01.x, wa);
    wa = fma(h01.y, x01.y, wa);
    wa = fma(h23.x, x23.x, wa);
    wa = fma(h23.y, x23.y, wa);
    wb = fma(g01.x, u01.x, wb);
    wb = fma(g01.y, u01.y, wb);
    wb = fma(g23.x, u23.x, wb);
    wb = fma(g23.y, u23.y, wb);
    if (S_TOO) {
      const double2 s01 = *reinterpret_cast<const double2*>(b0 + 16);
      const double2 s23 = *reinterpret_cast<const double2*>(b0 + 24);
      const double2 t01 = *reinterpret_cast<const double2*>(b1 + 16);
      const double2 t23 = *reinterpret_cast<const double2*>(b1 + 24);
      const double2 y01 = *reinterpret_cast<const double2*>(y + k0);
      const double2 y23 = *reinterpret_cast<const double2*>(y + k0 + 2);
      const double2 v01 = *reinterpret_cast<const double2*>(y + k1);
      const double2 v23 = *reinterpret_cast<const double2*>(y + k1 + 2);
      za = fma(s01.x, y01.x, za);
      za = fma(s01.y, y01.y, za);
      za = fma(s23.x, y23.x, za);
      za = fma(s23.y, y23.y, za);
      zb = fma(t01.x, v01.x, zb);
      zb = fma(t01.y, v01.y, zb);
      zb = fma(t23.x, v23.x, zb);
      zb = fma(t23.y, v23.y, zb);
    }
  }
  if (e < e1) {
    const unsigned p0 = s_ent[e];
    const double* b0 = rp + (p0 >> 8) * 32;
    const double2 h01 = *reinterpret_cast<const double2*>(b0);
    const double2 h23 = *reinterpret_cast<const double2*>(b0 + 8);
    const int k0 = NORB * (int)(p0 & 255);
    const double2 x01 = *reinterpret_cast<const double2*>(x + k0);
    const double2 x23 = *reinterpret_cast<const double2*>(x + k0 + 2);
    wa = fma(h01.x, x01.x, wa);
    wa = fma(h01.y, x01.y, wa);
    wa = fma(h23.x, x23.x, wa);
    wa = fma(h23.y, x23.y, wa);
    if (S_TOO) {
      const double2 s01 = *reinterpret_cast<const double2*>(b0 + 16);
      const double2 s23 = *reinterpret_cast<const double2*>(b0 + 24);
      const double2 y01 = *reinterpret_cast<const double2*>(y + k0);
      const double2 y23 = *reinterpret_cast<const double2*>(y + k0 + 2);
      za = fma(s01.x, y01.x, za);
      za = fma(s01.y, y01.y, za);
      za = fma(s23.x, y23.x, za);
      za = fma(s23.y, y23.y, za);
    }
  }
  hx = wa + wb;
  sy = za + zb;
}

// dot products of the basis columns 0 .. 8 (kc + 1) - 1 with v (rows held
// by this thread), plus |v|^2 when NORM: results in s_fin[0 ..] and
// s_fin[8 NCH]; the cross-wave sum is in a fixed order
template <int NU, int R, int KTPB, bool NORM>
__device__ __forceinline__ void basis_dots(const double (&qv)[R][NU], const double (&v)[R], int kc,
                                           double* s_red, double* s_fin) {
  constexpr int KWAVES = KTPB / 64;
  constexpr int NCH = (NU + 7) / 8;
  constexpr int RED = 8 * NCH + 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (c <= kc) {
      double t8[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int i = c * 8 + t;
        double p = 0.0;
        if (i < NU) {
#pragma unroll
          for (int rr = 0; rr < R; ++rr) p = fma(qv[rr][i], v[rr], p);
        }
        t8[t] = p;
      }
      const double r8 = reduce8(t8);
      if ((lane & 7) == 0) {
        const int idx = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
        s_red[wave * RED + c * 8 + idx] = r8;
      }
    }
  }
  if (NORM) {
    double ww = 0.0;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) ww = fma(v[rr], v[rr], ww);
    ww = wave_allreduce(ww);
    if (lane == 0) s_red[wave * RED + 8 * NCH] = ww;
  }
  __syncthreads();
  const int nval = 8 * (kc + 1);
  for (int t = threadIdx.x; t <= nval; t += KTPB) {
    if (t == nval && !NORM) break;
    const int tt = (t == nval) ? 8 * NCH : t;
    double acc = s_red[tt];
#pragma unroll
    for (int wv = 1; wv < KWAVES; ++wv) acc += s_red[wv * RED + tt];
    s_fin[tt] = acc;
  }
  __syncthreads();
}

// q_{cn} = w (register column cn) with uniform scalar branches on cn
template <int NU, int R>
__device__ __forceinline__ void store_column(double (&qv)[R][NU], const double (&w)[R], int cn) {
#pragma unroll
  for (int g = 0; g < (NU + 7) / 8; ++g) {
    if ((cn >> 3) == g) {
      __asm__ volatile("");
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int i = g * 8 + t;
        if (i >= 1 && i < NU && (cn & 7) == t) {
          __asm__ volatile("");
#pragma unroll
          for (int rr = 0; rr < R; ++rr) qv[rr][i] = w[rr];
        }
      }
    }
  }
}

// register column cn of the basis (uniform cn)
template <int NU, int R>
__device__ __forceinline__ void load_column(const double (&qv)[R][NU], double (&w)[R], int cn) {
#pragma unroll
  for (int rr = 0; rr < R; ++rr) w[rr] = 0.0;
#pragma unroll
  for (int i = 0; i < NU; ++i)
    if (i == cn) {
#pragma unroll
      for (int rr = 0; rr < R; ++rr) w[rr] = qv[rr][i];
    }
}

template <int NU, int R, int KTPB>
__global__ __launch_bounds__(KTPB) void adjoint_kernel(AdjointArgs a) {
  constexpr int NCH = (NU + 7) / 8;
  constexpr int RED = 8 * NCH + 8;
  constexpr int KWAVES = KTPB / 64;
  constexpr int KC = ADJ_KC;
  constexpr int NROW = KTPB * R;  // cluster rows the workgroup holds
  __shared__ int32_t s_atoms[CLUSTER_MAX];
  __shared__ int32_t s_lptr[CLUSTER_MAX + 1];
  __shared__ int32_t s_brow[CLUSTER_MAX];
  __shared__ int32_t s_gofs[CLUSTER_MAX + 1];
  __shared__ int32_t s_scan[KWAVES + 1];
  __shared__ uint16_t s_ent[AENT_MAX];
  __shared__ double s_pos[3 * CLUSTER_MAX];
  __shared__ double s_f[3 * CLUSTER_MAX];
  __shared__ double s_red[KWAVES * RED];
  __shared__ double s_fin[RED];
  __shared__ double s_beta[NU];
  __shared__ int s_misc[4];
  // dynamic: hbar, sbar (NU x NU each), then a region used by the sweep
  // (x, y, h, h hbar, c, v) and reused by the contraction (staged Q, Z)
  extern __shared__ double s_dyn[];
  double* s_hb = s_dyn;
  double* s_sb = s_hb + NU * NU;
  double* s_u = s_sb + NU * NU;
  double* s_x = s_u;
  double* s_y = s_x + NROW;
  double* s_h = s_y + NROW;
  double* s_hh = s_h + NU * NU;
  double* s_c = s_hh + NU * NU;
  double* s_v = s_c + NU * NU;
  double* s_sq = s_u;            // KC x NROW
  double* s_sz = s_u + KC * NROW;  // KC x NROW

  const int tid = threadIdx.x;
  const int cap = a.cap;
  const Box box{{a.box[0], a.box[1], a.box[2]}};
  // reciprocals for the contraction's minimum images and cutoff window
  const double ibx = 1.0 / box.L[0], iby = 1.0 / box.L[1], ibz = 1.0 / box.L[2];
  const double iw = 1.0 / (a.m.r_cut - a.m.r_on);
  // workgroup scratch: Wbar (then Z), Zs and Q, each NU columns of NROW rows
  double* wbar = a.wbar + (int64_t)blockIdx.x * 3 * NU * NROW;
  double* zsb = wbar + NU * NROW;
  double* qsb = zsb + NU * NROW;

  for (;;) {
    if (tid == 0) s_misc[0] = atomicAdd(a.counter, 1);
    __syncthreads();
    const int64_t ia = s_misc[0];
    __syncthreads();
    if (ia >= a.natoms) break;
    const int j0 = a.cols[4 * ia];
    const int J = j0 >> 2;
    bool ok = (j0 & 3) == 0;
    for (int al = 1; al < NORB; ++al) ok = ok && a.cols[4 * ia + al] == j0 + al;
    const int64_t c0 = a.clus_ptr[J];
    const int nat = (int)(a.clus_ptr[J + 1] - c0);
    const int nC = NORB * nat;
    if (!ok || nat > CLUSTER_MAX || nC > NROW || nat <= 0) {
      if (tid == 0) atomicOr(a.err, (int)(ok ? KERR_CAPACITY : KERR_LAYOUT));
      continue;
    }
    const int nbJ = a.bptr[J + 1] - a.bptr[J];

    // ---- cluster tables (the gather of H_C, S_C as a local block-CSR)
    int rlen = 0;
    for (int i = tid; i < nat; i += KTPB) {
      const int I = a.clus_atoms[c0 + i];
      const int b0 = a.bptr[I];
      s_atoms[i] = I;
      s_brow[i] = b0;
      rlen = a.bptr[I + 1] - b0;
      s_pos[3 * i] = a.pos[3 * (int64_t)I];
      s_pos[3 * i + 1] = a.pos[3 * (int64_t)I + 1];
      s_pos[3 * i + 2] = a.pos[3 * (int64_t)I + 2];
      s_f[3 * i] = 0.0;
      s_f[3 * i + 1] = 0.0;
      s_f[3 * i + 2] = 0.0;
    }
    int nflat = 0;
    const int gofs = adj_excl_scan<KTPB>(tid < nat ? rlen : 0, s_scan, &nflat);
    if (tid < nat) s_gofs[tid] = gofs;
    if (tid == 0) s_gofs[nat] = nflat;
    __syncthreads();
    const int chunk = (nflat + KTPB - 1) / KTPB;
    const int f0 = min(tid * chunk, nflat), f1 = min(f0 + chunk, nflat);
    int ia0 = 0;
    if (f0 < f1) {
      int lo = 0, hi = nat - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_gofs[mid] <= f0) lo = mid;
        else hi = mid - 1;
      }
      ia0 = lo;
    }
    int kept = 0;
    {
      int i = ia0;
      for (int f = f0; f < f1; ++f) {
        while (f >= s_gofs[i + 1]) ++i;
        const int b = s_brow[i] + (f - s_gofs[i]);
        if (adj_find(s_atoms, nat, a.bcol[b]) >= 0) ++kept;
      }
    }
    int nent = 0;
    int e = adj_excl_scan<KTPB>(kept, s_scan, &nent);
    if (tid == 0) {
      s_lptr[nat] = nent;
      s_misc[1] = adj_find(s_atoms, nat, J);
    }
    if (nent <= AENT_MAX) {
      int i = ia0;
      for (int f = f0; f < f1; ++f) {
        while (f >= s_gofs[i + 1]) ++i;
        const int off = f - s_gofs[i];
        if (off == 0) s_lptr[i] = e;
        const int b = s_brow[i] + off;
        const int kl = adj_find(s_atoms, nat, a.bcol[b]);
        if (kl >= 0) {
          s_ent[e] = (uint16_t)((off << 8) | kl);
          ++e;
        }
      }
    }
    __syncthreads();
    const int jl = s_misc[1];
    const int nbJl = (jl >= 0) ? s_lptr[jl + 1] - s_lptr[jl] : -1;
    if (nent > AENT_MAX || jl < 0 || nbJl != nbJ) {
      if (tid == 0) atomicOr(a.err, (int)(nent > AENT_MAX ? KERR_CAPACITY : KERR_PATTERN));
      __syncthreads();
      continue;
    }
    // row bookkeeping of this thread
    int e_beg[R], e_end[R];
    const double* rowp[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int r = R * tid + rr;
      e_beg[rr] = 0;
      e_end[rr] = 0;
      rowp[rr] = a.bval;
      if (r < nC) {
        e_beg[rr] = s_lptr[r >> 2];
        e_end[rr] = s_lptr[(r >> 2) + 1];
        rowp[rr] = a.bval + (int64_t)a.bptr[s_atoms[r >> 2]] * 32 + (r & 3) * 2;
      }
    }

    for (int alpha = 0; alpha < NORB; ++alpha) {
      const int64_t slot = 4 * ia + alpha;
      // ---- the forward pass's Krylov data of this column: its basis (in
      // registers, as the forward holds it), h, beta and the last residual
      const int n = a.nu_eff[slot];
      if (n < 1 || n > NU) continue;  // a failed column (the forward flagged it)
      double qv[R][NU];
      double rlast[R];
      {
        const double* qg = a.q + slot * (int64_t)cap * a.qrows;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          const int r = R * tid + rr;
          const bool in = r < nC;
#pragma unroll
          for (int k = 0; k < NU; ++k)
            qv[rr][k] = (in && k < n) ? qg[(int64_t)k * a.qrows + r] : 0.0;
          rlast[rr] = in ? a.r[slot * (int64_t)a.qrows + r] : 0.0;
        }
        const double* hg = a.h + slot * (int64_t)cap * cap;
        for (int idx = tid; idx < NU * NU; idx += KTPB) {
          const int i = idx / NU, k = idx - (idx / NU) * NU;
          const int lo = min(i, k), hi = max(i, k);
          s_h[idx] = (i < n && k < n) ? hg[(int64_t)hi * cap + lo] : 0.0;
        }
        for (int k = tid; k < NU; k += KTPB)
          s_beta[k] = (k + 1 < n) ? a.beta[slot * (int64_t)cap + k] : 0.0;
      }
      __syncthreads();

      // ---- the projected adjoints and the sweep's small matrices
      const double* hb_g = a.hbar + slot * (int64_t)(2 * cap * cap);
      for (int idx = tid; idx < NU * NU; idx += KTPB) {
        const int i = idx / NU, k = idx - (idx / NU) * NU;
        const bool in = i < n && k < n;
        s_hb[idx] = in ? hb_g[i * cap + k] : 0.0;
        s_sb[idx] = in ? hb_g[cap * cap + i * cap + k] : 0.0;
        if (!in) s_h[idx] = 0.0;
        s_c[idx] = 0.0;
      }
      __syncthreads();
      for (int idx = tid; idx < NU * NU; idx += KTPB) {
        const int p = idx / NU, i = idx - (idx / NU) * NU;
        double acc = 0.0;
        for (int m = 0; m < n; ++m) acc = fma(s_h[p * NU + m], s_hb[m * NU + i], acc);
        s_hh[idx] = acc;
      }
      double rb1[R], rb2[R], wb[R];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        rb1[rr] = 0.0;
        rb2[rr] = 0.0;
        wb[rr] = 0.0;
      }
      __syncthreads();

      // ---- reverse sweep over the steps k = n-2 .. 0 (step k made q_{k+1})
      for (int k = n - 2; k >= 0; --k) {
        const int i = k + 1;
        const bool has1 = i <= n - 2, has2 = i + 1 <= n - 2;
        // H operand: wbar_{i}; S operand: Q sbar e_i; Q coefficients v
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          const int r = R * tid + rr;
          double ys = 0.0;
#pragma unroll
          for (int m = 0; m < NU; ++m) ys = fma(qv[rr][m], s_sb[m * NU + i], ys);
          if (r < nC) {
            s_x[r] = wb[rr];
            s_y[r] = ys;
          }
        }
        for (int p = tid; p < NU; p += KTPB) {
          double acc = 2.0 * s_hh[p * NU + i];
          for (int m = i; m <= n - 2; ++m)
            if (p <= m + 1) acc = fma(-s_c[i * NU + m], s_h[p * NU + m], acc);
          s_v[p] = (p < n) ? acc : 0.0;
        }
        __syncthreads();
        const double al = s_h[i * NU + i];
        const double be = has2 ? s_h[i * NU + i + 1] : 0.0;
        const double hl = 2.0 * s_hb[(n - 1) * NU + i];
        double qb[R];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          double hx, sy;
          row_spmv<true>(rowp[rr], s_ent, e_beg[rr], e_end[rr], s_x, s_y, hx, sy);
          double acc = 0.0;
#pragma unroll
          for (int m = 0; m < NU; ++m) acc = fma(qv[rr][m], s_v[m], acc);
          acc = fma(hl, rlast[rr], acc);
          acc = fma(2.0, sy, acc);
          if (has1) acc += hx - al * rb1[rr];
          if (has2) acc = fma(-be, rb2[rr], acc);
          qb[rr] = (R * tid + rr < nC) ? acc : 0.0;
        }
        // p_m = q_m^T qbar for m <= i
        basis_dots<NU, R, KTPB, false>(qv, qb, i >> 3, s_red, s_fin);
        const double binv = 1.0 / s_beta[k];
        for (int m = tid; m <= k; m += KTPB) s_c[m * NU + k] = s_fin[m] * binv;
        double qi[R];
        load_column<NU, R>(qv, qi, i);
        const double pi_ = s_fin[i];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          double acc = qb[rr];
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            if (c <= (i >> 3)) {
#pragma unroll
              for (int t = 0; t < 8; ++t) {
                const int m = c * 8 + t;
                if (m < NU && m <= i) acc = fma(-qv[rr][m], s_fin[m], acc);
              }
            }
          }
          const double rbk = fma(-qi[rr], pi_, qb[rr]) * binv;
          const double wbk = acc * binv;
          rb2[rr] = rb1[rr];
          rb1[rr] = rbk;
          wb[rr] = wbk;
          const int r = R * tid + rr;
          if (r < NROW) wbar[(int64_t)k * NROW + r] = (r < nC) ? wbk : 0.0;
        }
        __syncthreads();
      }

      // ---- this thread's rows of Z = Wbar + Q hbar, Zs = Q sbar and Q, to
      // the workgroup's scratch (column k at k * NROW): the contraction
      // below reads them a few columns at a time, so the basis registers are
      // free there
      // (the basis columns go out first; Z and Zs are then formed from
      // them with the column index as a loop variable, not a register index)
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int r = R * tid + rr;
        if (r < NROW) {
#pragma unroll
          for (int k = 0; k < NU; ++k)
            if (k < n) qsb[(int64_t)k * NROW + r] = (r < nC) ? qv[rr][k] : 0.0;
        }
      }
      for (int k0 = 0; k0 < n; k0 += 8) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          const int r = R * tid + rr;
          if (r >= NROW) continue;
          double z[8], zs[8];
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) z[kk] = zs[kk] = 0.0;
          for (int m = 0; m < n; ++m) {
            const double qm = qsb[(int64_t)m * NROW + r];
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
              const int k = min(k0 + kk, NU - 1);
              z[kk] = fma(qm, s_hb[m * NU + k], z[kk]);
              zs[kk] = fma(qm, s_sb[m * NU + k], zs[kk]);
            }
          }
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            const int k = k0 + kk;
            if (k < n) {
              const int64_t o = (int64_t)k * NROW + r;
              if (k <= n - 2) z[kk] += wbar[o];
              wbar[o] = (r < nC) ? z[kk] : 0.0;
              zsb[o] = (r < nC) ? zs[kk] : 0.0;
            }
          }
        }
      }

      // ---- contraction with the Slater-Koster derivatives, KC basis
      // columns at a time
      double g3[R][3];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) g3[rr][0] = g3[rr][1] = g3[rr][2] = 0.0;
      for (int k0 = 0; k0 < n; k0 += KC) {
        {
          double zo[R][KC], zso[R][KC], qo[R][KC];
#pragma unroll
          for (int rr = 0; rr < R; ++rr) {
            const int r = R * tid + rr;
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
              const int k = k0 + kk;
              const bool in = k < n && r < NROW;
              const int64_t o = (int64_t)k * NROW + r;
              zo[rr][kk] = in ? wbar[o] : 0.0;
              zso[rr][kk] = in ? zsb[o] : 0.0;
              qo[rr][kk] = in ? qsb[o] : 0.0;
              if (r < NROW) {
                s_sq[kk * NROW + r] = qo[rr][kk];
                s_sz[kk * NROW + r] = zo[rr][kk];
              }
            }
          }
          __syncthreads();
#pragma unroll
          for (int rr = 0; rr < R; ++rr) {
            const int r = R * tid + rr;
            if (r < nC) {
              const int A = r >> 2, ar = r & 3;
              for (int e2 = e_beg[rr]; e2 < e_end[rr]; ++e2) {
                const int B = (int)(s_ent[e2] & 255);
                if (B == A) continue;
                double M[4] = {0.0, 0.0, 0.0, 0.0}, N[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                  const double2 q01 = *reinterpret_cast<const double2*>(s_sq + kk * NROW + 4 * B);
                  const double2 q23 = *reinterpret_cast<const double2*>(s_sq + kk * NROW + 4 * B + 2);
                  const double2 z01 = *reinterpret_cast<const double2*>(s_sz + kk * NROW + 4 * B);
                  const double2 z23 = *reinterpret_cast<const double2*>(s_sz + kk * NROW + 4 * B + 2);
                  const double zA = zo[rr][kk], qA = qo[rr][kk], sA = zso[rr][kk];
                  M[0] = fma(zA, q01.x, fma(qA, z01.x, M[0]));
                  M[1] = fma(zA, q01.y, fma(qA, z01.y, M[1]));
                  M[2] = fma(zA, q23.x, fma(qA, z23.x, M[2]));
                  M[3] = fma(zA, q23.y, fma(qA, z23.y, M[3]));
                  N[0] = fma(sA, q01.x, N[0]);
                  N[1] = fma(sA, q01.y, N[1]);
                  N[2] = fma(sA, q23.x, N[2]);
                  N[3] = fma(sA, q23.y, N[3]);
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) N[b] *= 2.0;
                double dx = s_pos[3 * B] - s_pos[3 * A], dy = s_pos[3 * B + 1] - s_pos[3 * A + 1],
                       dz = s_pos[3 * B + 2] - s_pos[3 * A + 2];
                dx -= box.L[0] * rint(dx * ibx);  // minimum image (|d| < r_cut < L / 2)
                dy -= box.L[1] * rint(dy * iby);
                dz -= box.L[2] * rint(dz * ibz);
                double gp[3];
                pair_row_grad(a.m, iw, dx, dy, dz, ar, M, N, gp);
                g3[rr][0] += gp[0];
                g3[rr][1] += gp[1];
                g3[rr][2] += gp[2];
              }
            }
          }
          __syncthreads();
        }
      }
      // the four rows of an atom are four neighbouring lanes (R = 1) or two
      // lanes (R = 2); sum them and let the first add to the atom's part
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double x = g3[rr][c];
          if (R == 1) {
            x += dpp_f64<DPP_QUAD_XOR1>(x);
            x += dpp_f64<DPP_QUAD_XOR2>(x);
          }
          g3[rr][c] = x;
        }
      }
      if (R == 1) {
        const int r = tid;
        if (r < nC && (r & 3) == 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) s_f[3 * (r >> 2) + c] += g3[0][c];
        }
      } else {
        // R = 2: rows 2t, 2t + 1 in one thread, the atom's other two rows in the neighbour lane
        double x[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          x[c] = g3[0][c] + g3[R - 1][c];
          x[c] += dpp_f64<DPP_QUAD_XOR1>(x[c]);
        }
        const int r = R * tid;
        if (r < nC && (r & 3) == 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) s_f[3 * (r >> 2) + c] += x[c];
        }
      }
      __syncthreads();
    }
    // ---- the atom's parts on its cluster atoms
    for (int idx = tid; idx < 3 * nat; idx += KTPB) a.fJ[3 * c0 + idx] = s_f[idx];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// stage 1: hbar, sbar of each column from its Ritz data (one wave per column)
__device__ __forceinline__ double omega_mu(double e, double mu, double kT) {
  const double x = (e - mu) / kT;
  return -kT * (fmax(-x, 0.0) + log1p(exp(-fabs(x))));
}

__device__ __forceinline__ double fermi_adj(double x) {
  if (x > 0.0) {
    const double e = exp(-x);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + exp(x));
}

// (omega(a) - omega(b)) / (a - b), omega' = f on the diagonal; for close
// arguments log1p(f_lo expm1(dx)) / dx, the exact integral of f over [lo, hi]
// written without cancellation
__device__ __forceinline__ double omega_dd(double ea, double eb, double mu, double kT) {
  const double lo = fmin(ea, eb), hi = fmax(ea, eb);
  const double xl = (lo - mu) / kT, xh = (hi - mu) / kT;
  const double dx = xl - xh;  // <= 0
  if (dx > -1.0) {
    const double fl = fermi_adj(xl);
    if (dx == 0.0) return fl;
    return log1p(fl * expm1(dx)) / dx;
  }
  return (omega_mu(lo, mu, kT) - omega_mu(hi, mu, kT)) / (lo - hi);
}

template <int NM>
__global__ __launch_bounds__(64) void adj_prep_kernel(const double* cvec, const double* cdg,
                                                      const int32_t* nu_eff, int64_t ncols,
                                                      const MuState* st, double* hbar) {
  extern __shared__ double sm[];
  constexpr int LD = NM + 1;
  double* C = sm;           // C[t][k]: component t of Ritz vector k
  double* M1 = C + NM * LD;  // K + K^T
  double* M2 = M1 + NM * LD;  // K Lambda + Lambda K^T
  double* T = M2 + NM * LD;   // M C^T
  const int64_t slot = blockIdx.x;
  if (slot >= ncols) return;
  const int lane = threadIdx.x;
  const int n = nu_eff[slot];
  double* out = hbar + slot * (int64_t)(2 * NM * NM);
  if (n <= 0 || n > NM) {
    for (int idx = lane; idx < 2 * NM * NM; idx += 64) out[idx] = 0.0;
    return;
  }
  const double mu = st->mu, kT = st->kT;
  const double* cv = cvec + slot * (int64_t)(NM * NM);
  const double* lam = cdg + slot * (int64_t)(3 * NM);
  const double* dv = lam + NM;
  const double* gv = dv + NM;
  for (int idx = lane; idx < NM * NM; idx += 64) {
    const int k = idx / NM, t = idx - (idx / NM) * NM;
    C[t * LD + k] = (t < n && k < n) ? cv[idx] : 0.0;
  }
  for (int idx = lane; idx < NM * NM; idx += 64) {
    const int p = idx / NM, q = idx - (idx / NM) * NM;
    double m1 = 0.0, m2 = 0.0;
    if (p < n && q < n) {
      const double lp = lam[p], lq = lam[q];
      const double D = omega_dd(lp, lq, mu, kT);
      const double kpq = D * dv[p] * gv[q], kqp = D * dv[q] * gv[p];
      m1 = kpq + kqp;
      m2 = kpq * lq + lp * kqp;
    }
    M1[p * LD + q] = m1;
    M2[p * LD + q] = m2;
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    const double* Mx = pass == 0 ? M1 : M2;
    for (int idx = lane; idx < NM * NM; idx += 64) {  // T[a][j] = sum_b M[a][b] C[j][b]
      const int p = idx / NM, q = idx - (idx / NM) * NM;
      double acc = 0.0;
      for (int b = 0; b < n; ++b) acc = fma(Mx[p * LD + b], C[q * LD + b], acc);
      T[p * LD + q] = acc;
    }
    __syncthreads();
    const double sgn = pass == 0 ? 1.0 : -1.0;
    for (int idx = lane; idx < NM * NM; idx += 64) {  // out[i][j] = sum_a C[i][a] T[a][j]
      const int i = idx / NM, q = idx - (idx / NM) * NM;
      double acc = 0.0;
      for (int b = 0; b < n; ++b) acc = fma(C[i * LD + b], T[b * LD + q], acc);
      out[pass * NM * NM + idx] = sgn * acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// stage 3: F_I = sum over the clusters holding I of their parts for I
__global__ void gather_forces_kernel(const int64_t* clus_ptr, const int32_t* clus_atoms,
                                     int64_t n, const double* fJ, double* F) {
  const int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (I >= n) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t q = clus_ptr[I]; q < clus_ptr[I + 1]; ++q) {
    const int J = clus_atoms[q];  // I lies in the cluster of J (the relation is symmetric)
    const int64_t b = clus_ptr[J];
    int lo = 0, hi = (int)(clus_ptr[J + 1] - b) - 1, pos = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int v = clus_atoms[b + mid];
      if (v == (int)I) {
        pos = mid;
        break;
      }
      if (v < (int)I) lo = mid + 1;
      else hi = mid - 1;
    }
    if (pos >= 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += fJ[3 * (b + pos) + c];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) F[3 * I + c] = acc[c];
}

// ---------------------------------------------------------------------------
// launchers
template <int NU, int R, int T>
static const void* afn() {
  return reinterpret_cast<const void*>(&adjoint_kernel<NU, R, T>);
}

struct AdjShape {
  int cap, tpb, r;
};
static const AdjShape kAdj[] = {{12, 768, 1}, {20, 768, 1}, {30, 768, 1}};

static const void* adj_fn(int cap) {
  switch (cap) {
    case 12: return afn<12, 1, 768>();
    case 20: return afn<20, 1, 768>();
    case 30: return afn<30, 1, 768>();
    default: return nullptr;
  }
}

int adjoint_supported(int cap) { return adj_fn(cap) != nullptr; }

size_t adjoint_dyn_lds(int cap) {
  for (const AdjShape& s : kAdj)
    if (s.cap == cap) {
      const size_t nrow = (size_t)s.tpb * s.r;
      const size_t sweep = 2 * nrow + 3 * (size_t)cap * cap + cap;
      const size_t stage = 2 * (size_t)ADJ_KC * nrow;
      return sizeof(double) * (2 * (size_t)cap * cap + std::max(sweep, stage));
    }
  return 0;
}

size_t adjoint_scratch_per_wg(int cap) {
  for (const AdjShape& s : kAdj)
    if (s.cap == cap) return sizeof(double) * 3 * (size_t)cap * s.tpb * s.r;
  return 0;
}

int adjoint_occupancy(int cap) {
  const void* fn = adj_fn(cap);
  if (!fn) return 0;
  const size_t dyn = adjoint_dyn_lds(cap);
  static bool set[64] = {};
  if (!set[cap]) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) !=
        hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    set[cap] = true;
  }
  int nb = 0;
  for (const AdjShape& s : kAdj)
    if (s.cap == cap &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, s.tpb, dyn) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
  return nb;
}

hipError_t launch_adjoint(const AdjointArgs& a, int grid, hipStream_t s) {
  const void* fn = adj_fn(a.cap);
  if (!fn || grid <= 0) return hipErrorInvalidValue;
  int tpb = 0;
  for (const AdjShape& sh : kAdj)
    if (sh.cap == a.cap) tpb = sh.tpb;
  AdjointArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(fn, dim3(grid), dim3(tpb), args, adjoint_dyn_lds(a.cap), s);
}

template <int NM>
static hipError_t launch_prep_nm(const double* cvec, const double* cdg, const int32_t* nu_eff,
                                 int64_t ncols, const MuState* st, double* hbar, hipStream_t s) {
  const size_t lds = sizeof(double) * 4 * NM * (NM + 1);
  hipLaunchKernelGGL(adj_prep_kernel<NM>, dim3((unsigned)ncols), dim3(64), lds, s, cvec, cdg,
                     nu_eff, ncols, st, hbar);
  return hipGetLastError();
}

hipError_t launch_adj_prep(const double* cvec, const double* cdg, const int32_t* nu_eff,
                           int64_t ncols, int cap, const MuState* st, double* hbar,
                           hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  switch (cap) {
    case 12: return launch_prep_nm<12>(cvec, cdg, nu_eff, ncols, st, hbar, s);
    case 20: return launch_prep_nm<20>(cvec, cdg, nu_eff, ncols, st, hbar, s);
    case 30: return launch_prep_nm<30>(cvec, cdg, nu_eff, ncols, st, hbar, s);
    case 40: return launch_prep_nm<40>(cvec, cdg, nu_eff, ncols, st, hbar, s);
    case 48: return launch_prep_nm<48>(cvec, cdg, nu_eff, ncols, st, hbar, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gather_forces(const int64_t* clus_ptr, const int32_t* clus_atoms, int64_t n,
                                const double* fJ, double* F, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_forces_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     clus_ptr, clus_atoms, n, fJ, F);
  return hipGetLastError();
}

}  // namespace mag
