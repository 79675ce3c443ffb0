// Per-column Krylov growth and projection (hot path of the multiple Arnoldi
// method: one Krylov subspace per column j of G = (zS - H)^-1, Eq. 1).
//
// One workgroup of KTPB threads owns one column j = (J, alpha) at a time.
// Its cluster C(J) is gathered in LDS as a local block-CSR over the global
// 4x4-block matrices (prologue), then nu Krylov steps run with the basis Q
// (n_C x nu) distributed over the registers of the workgroup: thread t owns
// cluster rows R t + r, r < R (so wave w always holds rows 64 R w .. 64 R w +
// 64 R - 1 and the results do not depend on the workgroup size).  Each step:
//   w = H_C q_k, z = S_C q_k       one fused SpMV (shared pattern and gathers)
//   h[:,k] = Q^T w, s[:,k] = Q^T z  projection, taken from the first
//                                   Gram-Schmidt pass's dot products
//   w -= Q h[:,k]; c = Q^T w; w -= Q c   classical Gram-Schmidt; the second
//                                        pass runs when the first one removed
//                                        more than half of |w|^2
//   q_{k+1} = w / |w|                    (breakdown: |w| <= tol |H q_k|)
// The basis is Euclidean-orthonormal; it spans the same Krylov space
// K_nu(H_C; e_l) as the S-orthonormal basis of the method's reading, so the
// projected pencil (h, s) has the same Ritz pairs.  Dot products are reduced
// with a deterministic wave reduce-scatter plus a fixed-order cross-wave sum,
// so a column's result does not depend on which workgroup computes it.
//
// Scheduling: persistent workgroups pull columns from KRYLOV_QUEUES device
// queues, each a spatially compact range of atoms; workgroup w starts on
// queue w % KRYLOV_QUEUES (workgroups are dealt to the XCDs round-robin, so a
// queue's clusters share that XCD's L2) and steals from the others when its
// own is empty.
#include <algorithm>
#include <cstdlib>

#include "mag_internal.h"
#include "wave.h"

namespace mag {

constexpr int ENT_MAX = CLUSTER_MAX * 24;  // local blocks of a cluster
constexpr int CACHE_MAX = 640;             // cluster blocks held in LDS at most
constexpr int CSLOT = CSLOT_BYTES / 16;    // double2 per cached block (16 + bank pad)

// exclusive prefix sum of one int per thread over the workgroup (s_scan: one
// int per wave plus one); returns the thread's offset, *total the sum
template <int KTPB>
__device__ __forceinline__ int block_excl_scan(int v, int32_t* s_scan, int* total) {
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

// one row of a 4x4 H block and of the S block against the block column's x
#define MAG_BLOCK_FMA1                 \
  wa = fma(h01.x, x01.x, wa);          \
  wa = fma(h01.y, x01.y, wa);          \
  wa = fma(h23.x, x23.x, wa);          \
  wa = fma(h23.y, x23.y, wa);          \
  za = fma(s01.x, x01.x, za);          \
  za = fma(s01.y, x01.y, za);          \
  za = fma(s23.x, x23.x, za);          \
  za = fma(s23.y, x23.y, za);
// two blocks, the second into separate accumulators
#define MAG_BLOCK_FMA                  \
  MAG_BLOCK_FMA1                       \
  wb = fma(g01.x, y01.x, wb);          \
  wb = fma(g01.y, y01.y, wb);          \
  wb = fma(g23.x, y23.x, wb);          \
  wb = fma(g23.y, y23.y, wb);          \
  zb = fma(t01.x, y01.x, zb);          \
  zb = fma(t01.y, y01.y, zb);          \
  zb = fma(t23.x, y23.x, zb);          \
  zb = fma(t23.y, y23.y, zb);

// the same for named operands: accumulators (wacc, zacc), the block's H and S
// rows, and x of the block column
#define MAG_ROW_FMA(wacc, zacc, h01, h23, s01, s23, x01, x23) \
  wacc = fma(h01.x, x01.x, wacc);                           \
  wacc = fma(h01.y, x01.y, wacc);                           \
  wacc = fma(h23.x, x23.x, wacc);                           \
  wacc = fma(h23.y, x23.y, wacc);                           \
  zacc = fma(s01.x, x01.x, zacc);                           \
  zacc = fma(s01.y, x01.y, zacc);                           \
  zacc = fma(s23.x, x23.x, zacc);                           \
  zacc = fma(s23.y, x23.y, zacc);

template <int NU, int R, int KTPB, bool ADJ>
__global__ __launch_bounds__(KTPB) void krylov_kernel(KrylovArgs a) {
  constexpr int KWAVES = KTPB / 64;
  constexpr int NCH = (NU + 7) / 8;
  constexpr int RED = 16 * NCH + 8;
  __shared__ int32_t s_atoms[CLUSTER_MAX];
  __shared__ int32_t s_lptr[CLUSTER_MAX + 1];
  __shared__ int32_t s_brow[CLUSTER_MAX];      // first global block of each cluster atom's row
  __shared__ int32_t s_gofs[CLUSTER_MAX + 1];  // offsets of those rows in the flattened list
  __shared__ int32_t s_scan[KTPB / 64 + 1];
  // local block-CSR entry: (block offset in the global block row << 8) | local column atom
  __shared__ uint16_t s_ent[ENT_MAX];
  __shared__ int32_t s_cblk[CACHE_MAX];  // global block of each cached entry
  // the first H and S blocks of the cluster (prefix of the entry list), kept for
  // all nu steps of the column
  extern __shared__ double2 s_cache[];
  __shared__ int16_t s_pat[NC_MAX];
  __shared__ double s_x[NC_MAX];
  __shared__ double s_red[KWAVES][RED];
  __shared__ double s_fin[RED];
  __shared__ int s_misc[4];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cap = a.cap;
  int q = a.queue ? (int)(blockIdx.x % (unsigned)a.nqueue) : 0;
  int tried = 0;
  // a queue hands out the NORB columns of an atom together while more than
  // `tail` columns remain in it, and single columns after that; the columns
  // of one atom share the cluster tables built by the prologue
  const int64_t tail = a.queue ? (int64_t)NORB * (gridDim.x / a.nqueue + 1) : 0;
  int tabJ = -1;  // atom whose cluster tables the LDS holds (-1: none)
  int tab_jl = 0, tab_ncache = 0;

  for (int64_t it = 0;; ++it) {
    int64_t base;
    int count;
    if (a.queue) {
      if (tid == 0) {
        int64_t sl = -1;
        int n = 0;
        while (tried < a.nqueue) {
          const int64_t qb = a.qbeg[q], qe = a.qbeg[q + 1];
          const int64_t seen = qb + atomicAdd(&a.queue[q], 0);
          const int g = (qe - seen > tail) ? NORB : 1;
          const int64_t cand = qb + atomicAdd(&a.queue[q], g);
          if (cand < qe) {
            sl = cand;
            n = (int)min((int64_t)g, qe - cand);
            break;
          }
          q = (q + 1) % a.nqueue;
          ++tried;
        }
        s_misc[0] = (int)sl;
        s_misc[2] = n;
      }
      __syncthreads();
      base = s_misc[0];
      count = s_misc[2];
      __syncthreads();
      if (base < 0) break;
    } else {
      if (it > 0) break;
      base = blockIdx.x;
      count = 1;
    }
    if (base >= a.ncols) break;

    for (int u = 0; u < count; ++u) {
      int64_t slot = base + u;
      if (a.slots) slot = a.slots[slot];  // this launch covers a subset of the slots

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
      const int nbJ = a.bptr[J + 1] - a.bptr[J];

      if (J != tabJ) {
        // ---- prologue: cluster atoms and local block rows (gather of H_C, S_C).
        // The global block rows of the cluster atoms are flattened into one
        // list; each thread tests a contiguous chunk of it for cluster
        // membership (binary search in the sorted atoms), and a workgroup scan
        // of the kept counts places the local entries in CSR order.
        tabJ = -1;
        int rlen = 0;
        for (int i = tid; i < nat; i += KTPB) {
          const int I = a.clus_atoms[c0 + i];
          const int b0 = a.bptr[I];
          s_atoms[i] = I;
          s_brow[i] = b0;
          rlen = a.bptr[I + 1] - b0;
        }
        for (int i = tid; i < nC; i += KTPB) s_pat[i] = -1;
        int nflat = 0;
        const int gofs = block_excl_scan<KTPB>(tid < nat ? rlen : 0, s_scan, &nflat);
        if (tid < nat) s_gofs[tid] = gofs;
        if (tid == 0) s_gofs[nat] = nflat;
        __syncthreads();
        const int chunk = (nflat + KTPB - 1) / KTPB;
        const int f0 = min(tid * chunk, nflat), f1 = min(f0 + chunk, nflat);
        // atom of the chunk's first flat entry
        int ia = 0;
        if (f0 < f1) {
          int lo = 0, hi = nat - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_gofs[mid] <= f0) lo = mid;
            else hi = mid - 1;
          }
          ia = lo;
        }
        int kept = 0;
        {
          int i = ia;
          for (int f = f0; f < f1; ++f) {
            while (f >= s_gofs[i + 1]) ++i;
            const int b = s_brow[i] + (f - s_gofs[i]);
            if (lds_find(s_atoms, nat, a.bcol[b]) >= 0) ++kept;
          }
        }
        int nent = 0;
        int e = block_excl_scan<KTPB>(kept, s_scan, &nent);
        if (tid == 0) {
          s_lptr[nat] = nent;
          s_misc[1] = lds_find(s_atoms, nat, J);
        }
        const int ncache = min(nent, a.cache_cap);
        if (nent <= ENT_MAX) {
          int i = ia;
          for (int f = f0; f < f1; ++f) {
            while (f >= s_gofs[i + 1]) ++i;
            const int off = f - s_gofs[i];
            if (off == 0) s_lptr[i] = e;  // first flat entry of atom i's row
            const int b = s_brow[i] + off;
            const int kl = lds_find(s_atoms, nat, a.bcol[b]);
            if (kl >= 0) {
              s_ent[e] = (uint16_t)((off << 8) | kl);
              if (e < ncache) s_cblk[e] = b;
              ++e;
            }
          }
        }
        __syncthreads();
        const int jl = s_misc[1];
        const int nbJl = (jl >= 0) ? s_lptr[jl + 1] - s_lptr[jl] : -1;
        if (nent > ENT_MAX || jl < 0 || nbJl != nbJ) {
          if (tid == 0) {
            atomicOr(a.err, (int)(nent > ENT_MAX ? KERR_CAPACITY : KERR_PATTERN));
            a.nu_eff[slot] = 0;
          }
          __syncthreads();
          continue;
        }
        // pattern rows of column j: block row of J, in CSR order (block t, orbital)
        for (int t = tid; t < NORB * nbJ; t += KTPB) {
          const int kl = (int)(s_ent[s_lptr[jl] + (t >> 2)] & 255);
          s_pat[NORB * kl + (t & 3)] = (int16_t)t;
        }
        // cached entry e sits at e * 17 double2 (272 bytes): the 16-byte pad puts
        // consecutive atoms of a wave on different LDS bank groups
        {
          const double2* bv2 = reinterpret_cast<const double2*>(a.bval);
          for (int idx = tid; idx < ncache * 16; idx += KTPB)
            s_cache[(idx >> 4) * CSLOT + (idx & 15)] = bv2[(int64_t)s_cblk[idx >> 4] * 16 + (idx & 15)];
        }
        tabJ = J;
        tab_jl = jl;
        tab_ncache = ncache;
      }
      const int jl = tab_jl;
      const int ncache = tab_ncache;
      const int ell = NORB * jl + alpha;
      for (int i = tid; i < nC; i += KTPB) s_x[i] = (i == ell) ? 1.0 : 0.0;

      double qv[R][NU];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
#pragma unroll
        for (int i = 0; i < NU; ++i) qv[rr][i] = 0.0;
        if (R * tid + rr == ell) qv[rr][0] = 1.0;
      }
      // row bookkeeping of this thread: entry range, the split between cached
      // and streamed blocks, and the row's position inside its global blocks
      int e_beg[R], e_mid[R], e_end[R], r_off[R];
      const double* rowp[R];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int r = R * tid + rr;
        e_beg[rr] = 0;
        e_end[rr] = 0;
        r_off[rr] = (r & 3) * 2;  // row a of a block: doubles 2a, 2a+1 of each 8-double quarter
        rowp[rr] = a.bval;
        if (r < nC) {
          e_beg[rr] = s_lptr[r >> 2];
          e_end[rr] = s_lptr[(r >> 2) + 1];
          rowp[rr] = a.bval + (int64_t)a.bptr[s_atoms[r >> 2]] * 32 + r_off[rr];
        }
        e_mid[rr] = min(max(ncache, e_beg[rr]), e_end[rr]);
      }
      const int nu_max = min(a.nu, nC);
      int nu_eff = nu_max;
      double* hcol = a.hs + slot * (int64_t)(2 * cap * cap);
      double* scol = hcol + cap * cap;
      __syncthreads();

      for (int k = 0; k < nu_max; ++k) {
        // ---- fused SpMV: w = H_C q_k, z = S_C q_k (two blocks per iteration);
        // cached blocks come from LDS, the rest stream from L2/HBM
        double w[R], z[R];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          double wa = 0.0, za = 0.0, wb = 0.0, zb = 0.0;
          const int ro = r_off[rr];
          int e = e_beg[rr];
          const int em = e_mid[rr], e1 = e_end[rr];
          for (; e + 1 < em; e += 2) {
            const double2* c0p = s_cache + e * CSLOT + (ro >> 1);
            const double2* c1p = c0p + CSLOT;
            const double2 h01 = c0p[0], h23 = c0p[4], s01 = c0p[8], s23 = c0p[12];
            const double2 g01 = c1p[0], g23 = c1p[4], t01 = c1p[8], t23 = c1p[12];
            const int k0 = NORB * (s_ent[e] & 255), k1 = NORB * (s_ent[e + 1] & 255);
            const double2 x01 = *reinterpret_cast<const double2*>(s_x + k0);
            const double2 x23 = *reinterpret_cast<const double2*>(s_x + k0 + 2);
            const double2 y01 = *reinterpret_cast<const double2*>(s_x + k1);
            const double2 y23 = *reinterpret_cast<const double2*>(s_x + k1 + 2);
            MAG_BLOCK_FMA
          }
          if (e < em) {
            const double2* c0p = s_cache + e * CSLOT + (ro >> 1);
            const double2 h01 = c0p[0], h23 = c0p[4], s01 = c0p[8], s23 = c0p[12];
            const int k0 = NORB * (s_ent[e] & 255);
            const double2 x01 = *reinterpret_cast<const double2*>(s_x + k0);
            const double2 x23 = *reinterpret_cast<const double2*>(s_x + k0 + 2);
            MAG_BLOCK_FMA1
            ++e;
          }
          // entries alternate between the two accumulator pairs by their
          // offset in the row, so each pair sums the same blocks in the same
          // order wherever the cached part ends (the result does not depend
          // on the cache size of the launch plan): continue with the pair
          // that the next offset's parity names, and swap after an odd
          // number of entries
          if ((e - e_beg[rr]) & 1) {
            const double tw = wa, tz = za;
            wa = wb;
            za = zb;
            wb = tw;
            zb = tz;
          }
          // streamed blocks, three per iteration (twelve loads in flight)
          const double* rp = rowp[rr];
          for (; e + 2 < e1; e += 3) {
            double2 h01[3], h23[3], s01[3], s23[3];
            int kk[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
              const unsigned p = s_ent[e + u];
              const double* b = rp + (p >> 8) * 32;
              h01[u] = *reinterpret_cast<const double2*>(b);
              h23[u] = *reinterpret_cast<const double2*>(b + 8);
              s01[u] = *reinterpret_cast<const double2*>(b + 16);
              s23[u] = *reinterpret_cast<const double2*>(b + 24);
              kk[u] = NORB * (int)(p & 255);
            }
#pragma unroll
            for (int u = 0; u < 3; ++u) {
              const double2 x01 = *reinterpret_cast<const double2*>(s_x + kk[u]);
              const double2 x23 = *reinterpret_cast<const double2*>(s_x + kk[u] + 2);
              if (u == 1) {
                MAG_ROW_FMA(wb, zb, h01[u], h23[u], s01[u], s23[u], x01, x23)
              } else {
                MAG_ROW_FMA(wa, za, h01[u], h23[u], s01[u], s23[u], x01, x23)
              }
            }
            const double tw = wa, tz = za;  // three entries: the parity flips
            wa = wb;
            za = zb;
            wb = tw;
            zb = tz;
          }
          for (; e < e1; ++e) {
            const unsigned p0 = s_ent[e];
            const double* b0 = rp + (p0 >> 8) * 32;
            const double2 h01 = *reinterpret_cast<const double2*>(b0);
            const double2 h23 = *reinterpret_cast<const double2*>(b0 + 8);
            const double2 s01 = *reinterpret_cast<const double2*>(b0 + 16);
            const double2 s23 = *reinterpret_cast<const double2*>(b0 + 24);
            const int k0 = NORB * (p0 & 255);
            const double2 x01 = *reinterpret_cast<const double2*>(s_x + k0);
            const double2 x23 = *reinterpret_cast<const double2*>(s_x + k0 + 2);
            MAG_ROW_FMA(wa, za, h01, h23, s01, s23, x01, x23)
            const double tw = wa, tz = za;
            wa = wb;
            za = zb;
            wb = tw;
            zb = tz;
          }
          w[rr] = wa + wb;  // the same sum in either order
          z[rr] = za + zb;
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
                  ph = fma(qv[rr][i], w[rr], ph);
                  ps = fma(qv[rr][i], z[rr], ps);
                }
              }
              v[t] = ph;
              v[8 + t] = ps;
            }
            const double r16 = reduce16(v);
            if ((lane & 3) == 0) {
              const int idx = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 +
                              ((lane >> 2) & 1) * 2 + ((lane >> 3) & 1);
              s_red[wave][c * 16 + idx] = r16;
            }
          }
        }
        {
          double ww = 0.0;
#pragma unroll
          for (int rr = 0; rr < R; ++rr) ww = fma(w[rr], w[rr], ww);
          ww = wave_allreduce(ww);
          if (lane == 0) s_red[wave][16 * NCH] = ww;
        }
        __syncthreads();
        {
          const int nval = 16 * (kc + 1);
          for (int t = tid; t <= nval; t += KTPB) {
            const int tt = (t == nval) ? 16 * NCH : t;
            double acc = s_red[0][tt];
#pragma unroll
            for (int wv = 1; wv < KWAVES; ++wv) acc += s_red[wv][tt];
            s_fin[tt] = acc;
          }
        }
        __syncthreads();
        const double ww1 = s_fin[16 * NCH];
        for (int i = tid; i <= k; i += KTPB) {
          hcol[(int64_t)k * cap + i] = s_fin[(i >> 3) * 16 + (i & 7)];
          scol[(int64_t)k * cap + i] = s_fin[(i >> 3) * 16 + 8 + (i & 7)];
          if (ADJ) a.adj_h[slot * (int64_t)cap * cap + (int64_t)k * cap + i] =
              s_fin[(i >> 3) * 16 + (i & 7)];
        }
        // a single exit at the bottom of the step keeps the basis registers in
        // place (each early exit would need its own copy of them)
        bool go = (k + 1 < nu_max);
        bool orth = false;  // w orthogonalized in this step
        if (!isfinite(ww1)) {
          if (tid == 0) atomicOr(a.err, (int)KERR_NONFINITE);
          nu_eff = k + 1;
          go = false;
        }
        if (go) {
        orth = true;

        // ---- w -= Q h[:, k]; |h|^2 rides along (columns past k hold zeros)
        double hsq = 0.0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          if (c <= kc) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const int i = c * 8 + t;
              if (i < NU) {
                const double hi = s_fin[c * 16 + t];
                hsq = fma(hi, hi, hsq);
#pragma unroll
                for (int rr = 0; rr < R; ++rr) w[rr] = fma(-qv[rr][i], hi, w[rr]);
              }
            }
          }
        }
        // second pass c = Q^T w, w -= Q c only when the first pass cancelled
        // more than half of |w|^2 (the criterion of Daniel, Gragg, Kaufman and
        // Stewart, eta = 1/sqrt 2); otherwise |w|^2 - |h|^2 is the new norm^2
        double beta2 = ww1 - hsq;
        if (!(beta2 > 0.5 * ww1)) {
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
                  for (int rr = 0; rr < R; ++rr) p = fma(qv[rr][i], w[rr], p);
                }
                v[t] = p;
              }
              const double r8 = reduce8(v);
              if ((lane & 7) == 0) {
                const int idx = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
                s_red[wave][c * 8 + idx] = r8;
              }
            }
          }
          {
            double ww = 0.0;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) ww = fma(w[rr], w[rr], ww);
            ww = wave_allreduce(ww);
            if (lane == 0) s_red[wave][8 * NCH] = ww;
          }
          __syncthreads();
          {
            const int nval = 8 * (kc + 1);
            for (int t = tid; t <= nval; t += KTPB) {
              const int tt = (t == nval) ? 8 * NCH : t;
              double acc = s_red[0][tt];
#pragma unroll
              for (int wv = 1; wv < KWAVES; ++wv) acc += s_red[wv][tt];
              s_fin[tt] = acc;
            }
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
                  for (int rr = 0; rr < R; ++rr) w[rr] = fma(-qv[rr][i], ci, w[rr]);
                }
              }
            }
          }
          beta2 = s_fin[8 * NCH] - csq;
          if (!(beta2 > 0.5 * s_fin[8 * NCH])) {
            // the second pass removed a large part: take the norm explicitly
            __syncthreads();
            double ww = 0.0;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) ww = fma(w[rr], w[rr], ww);
            ww = wave_allreduce(ww);
            if (lane == 0) s_red[wave][0] = ww;
            __syncthreads();
            double acc = s_red[0][0];
#pragma unroll
            for (int wv = 1; wv < KWAVES; ++wv) acc += s_red[wv][0];
            beta2 = acc;
          }
        }
        // breakdown: |w| <= tol |H q_k|, compared in squares
        const double b2 = fmax(beta2, 0.0);
        if (!(b2 > a.breakdown * a.breakdown * ww1)) {
          nu_eff = k + 1;
          go = false;
        } else {
          const double inv = rsqrt(b2);
          if (ADJ && tid == 0) a.adj_beta[slot * (int64_t)cap + k] = sqrt(b2);
#pragma unroll
          for (int rr = 0; rr < R; ++rr) w[rr] *= inv;
          // q_{k+1} into its register column.  k is uniform, so each test is a
          // scalar branch: first the group of eight columns, then the column
          // inside it (a dozen scalar tests instead of one per column; the
          // empty asm statements keep the compiler from turning the tests into
          // selects or a switch whose merge copies every column)
          const int cn = k + 1;
#pragma unroll
          for (int g = 0; g < (NU + 7) / 8; ++g) {
            if ((cn >> 3) == g) {
              __asm__ volatile("");
#pragma unroll
              for (int t = 0; t < 8; ++t) {
                const int i = g * 8 + t;
                if (i >= 1 && i < NU && (cn & 7) == t) {
                  __asm__ volatile("");  // keep the branch (no speculation into selects)
#pragma unroll
                  for (int rr = 0; rr < R; ++rr) qv[rr][i] = w[rr];
                }
              }
            }
          }
#pragma unroll
          for (int rr = 0; rr < R; ++rr) {
            const int r = R * tid + rr;
            if (r < nC) s_x[r] = w[rr];
          }
        }
        }
        if (ADJ && !go) {
          // the last step's residual H q_n - Q h[:, n-1] for the exact
          // gradient (a breakdown step has already orthogonalized w)
          if (!orth) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
              if (c <= kc) {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                  const int i = c * 8 + t;
                  if (i < NU) {
                    const double hi = s_fin[c * 16 + t];
#pragma unroll
                    for (int rr = 0; rr < R; ++rr) w[rr] = fma(-qv[rr][i], hi, w[rr]);
                  }
                }
              }
            }
          }
#pragma unroll
          for (int rr = 0; rr < R; ++rr) {
            const int r = R * tid + rr;
            if (r < a.adj_rows) a.adj_r[slot * (int64_t)a.adj_rows + r] = (r < nC) ? w[rr] : 0.0;
          }
        }
        __syncthreads();
        if (!go) break;
      }

      // ---- epilogue: nu_eff, row l of Q, and the pattern (or all) rows of Q
      if (tid == 0) {
        a.nu_eff[slot] = nu_eff;
        if (a.npat) a.npat[slot] = a.full ? nC : NORB * nbJ;
      }
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int r = R * tid + rr;
        if (r < nC) {
          if (r == ell) {
            double* u = a.urow + slot * (int64_t)cap;
#pragma unroll
            for (int i = 0; i < NU; ++i) u[i] = qv[rr][i];
            for (int i = NU; i < cap; ++i) u[i] = 0.0;
          }
          const int p = a.full ? r : (int)s_pat[r];
          if (p >= 0) {
            double* dst = a.qpat + (slot * (int64_t)a.pat_stride + p) * cap;
#pragma unroll
            for (int i = 0; i < NU; ++i) dst[i] = qv[rr][i];
            for (int i = NU; i < cap; ++i) dst[i] = 0.0;
          }
        }
        if (ADJ && r < a.adj_rows) {
          double* dq = a.adj_q + slot * (int64_t)cap * a.adj_rows + r;
#pragma unroll
          for (int i = 0; i < NU; ++i) dq[(int64_t)i * a.adj_rows] = (r < nC) ? qv[rr][i] : 0.0;
        }
      }
      __syncthreads();
    }
  }
}

// Workgroup shapes.  nu <= 30 keeps one cluster row per thread (up to 168
// VGPRs: three waves per SIMD); 256-, 512- and 768-thread workgroups hold
// clusters of up to 64, 128 and 192 atoms.  nu = 40, 48 have two-row shapes
// (256 and 512 threads) and a one-row 768-thread shape whose basis does not
// fit the 168 registers and partly spills: on the void cell's large clusters
// it still runs 1.3-1.4 times faster than the two-row shape that holds them.
// nu = 30 also has a 640-thread shape (clusters up to 160 atoms, ten waves:
// no idle waves in the dots and barriers for the 141-160-atom clusters of a
// 6 A cutoff in diamond).  The library picks a shape per bucket of cluster
// sizes and times every shape that holds the bucket once (see run_columns).  Shapes with one and with two rows per
// thread add a thread's rows in a different grouping, so for nu = 40, 48 a
// column's last bits depend on the plan chosen; every launch of a context
// keeps its plans.
template <int NU, int R, int T>
static const void* kfn(bool adj) {
  return adj ? reinterpret_cast<const void*>(&krylov_kernel<NU, R, T, true>)
             : reinterpret_cast<const void*>(&krylov_kernel<NU, R, T, false>);
}

static const KrylovShapeInfo kShapes[] = {
    {12, 256, 1, nullptr}, {12, 512, 1, nullptr}, {12, 768, 1, nullptr},
    {20, 256, 1, nullptr}, {20, 512, 1, nullptr}, {20, 768, 1, nullptr},
    {30, 256, 1, nullptr}, {30, 512, 1, nullptr}, {30, 768, 1, nullptr},
    {40, 256, 2, nullptr}, {40, 512, 2, nullptr},
    {48, 256, 2, nullptr}, {48, 512, 2, nullptr},
    {40, 768, 1, nullptr}, {48, 768, 1, nullptr},
    {30, 640, 1, nullptr},
};
constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));

// the kernel of shape `id`; adj: the variant that also leaves each column's
// basis, h, beta and last residual for the exact gradient (nu <= 30 shapes only)
static const void* shape_fn(int id, bool adj = false) {
  switch (id) {
    case 0: return kfn<12, 1, 256>(adj);
    case 1: return kfn<12, 1, 512>(adj);
    case 2: return kfn<12, 1, 768>(adj);
    case 3: return kfn<20, 1, 256>(adj);
    case 4: return kfn<20, 1, 512>(adj);
    case 5: return kfn<20, 1, 768>(adj);
    case 6: return kfn<30, 1, 256>(adj);
    case 7: return kfn<30, 1, 512>(adj);
    case 8: return kfn<30, 1, 768>(adj);
    case 9: return adj ? nullptr : kfn<40, 2, 256>(false);
    case 10: return adj ? nullptr : kfn<40, 2, 512>(false);
    case 11: return adj ? nullptr : kfn<48, 2, 256>(false);
    case 12: return adj ? nullptr : kfn<48, 2, 512>(false);
    case 13: return adj ? nullptr : kfn<40, 1, 768>(false);
    case 14: return adj ? nullptr : kfn<48, 1, 768>(false);
    case 15: return kfn<30, 1, 640>(adj);
    default: return nullptr;
  }
}

int krylov_shapes(int cap, KrylovShapeInfo* out, int max_out) {
  int n = 0;
  for (int i = 0; i < kNumShapes; ++i) {
    if (kShapes[i].cap != cap) continue;
    if (n < max_out) {
      out[n] = kShapes[i];
      out[n].id = i;
    }
    ++n;
  }
  return n;
}

size_t krylov_static_lds(int id) {
  hipFuncAttributes attr{};
  if (hipFuncGetAttributes(&attr, shape_fn(id)) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return attr.sharedSizeBytes;
}

// cached blocks that `dyn` bytes of dynamic LDS hold
int krylov_cache_blocks(size_t dyn) {
  return std::min<int>(CACHE_MAX, (int)(dyn / (CSLOT * sizeof(double2))));
}

// workgroups of shape `id` that fit on one CU with `dyn` bytes of dynamic
// LDS each (0 if the launch would not fit); also raises the kernel's dynamic
// LDS limit to `dyn`
int krylov_occupancy(int id, size_t dyn) {
  const void* fn = shape_fn(id);
  if (!fn) return 0;
  // the kernel's dynamic LDS limit only ever rises, so a query never lowers
  // it below what an earlier plan launches with
  static size_t dyn_set[kNumShapes] = {};
  if (dyn > dyn_set[id]) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) !=
        hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    // the exact-gradient variant launches with the same plans
    const void* fa = shape_fn(id, true);
    if (fa && hipFuncSetAttribute(fa, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) !=
                  hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    dyn_set[id] = dyn;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kShapes[id].tpb, dyn) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

hipError_t launch_krylov(const KrylovArgs& a, int id, size_t dyn, int grid, hipStream_t s) {
  const void* fn = shape_fn(id, a.adj_q != nullptr);
  if (!fn || grid <= 0) return hipErrorInvalidValue;
  KrylovArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(fn, dim3(grid), dim3(kShapes[id].tpb), args, dyn, s);
}

int krylov_capacity(int nu) {
  static const int caps[] = {12, 20, 30, 40, 48};
  for (int c : caps)
    if (nu <= c) return c;
  return 0;
}

}  // namespace mag
