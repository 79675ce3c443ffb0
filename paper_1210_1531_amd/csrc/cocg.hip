// Green's-function columns by COCG on the column's cluster (a second solver
// of the generalized shifted equation (z S - H) x = b, Eq. 1).
//
// For real symmetric H and S and complex z, A = z S - H is complex symmetric,
// and the conjugate orthogonal conjugate gradient method of van der Vorst and
// Melissen is CG with the bilinear form <u, v> = u^T v.  Column j = (J, alpha)
// solves A_C x = e_l on the cluster of atom J (A_C = z S_C - H_C, the same
// locality as the multiple Arnoldi columns), so the result is the column of
// (z S_C - H_C)^-1; for a whole-cell cluster it is the column of (z S - H)^-1.
//
// One workgroup per column, one cluster row per thread.  The cluster's local
// block-CSR (entries into the global 4x4-block rows) is built in LDS; each
// iteration reads the row's H and S blocks once and applies them to the
// search directions of CG_NZ energies together, so the matrix traffic is
// shared by the energies.  Reductions are per-wave all-reduces plus a
// fixed-order cross-wave sum, so every thread sees the same sums and the
// per-energy control flow is uniform across the workgroup.
#include "mag_internal.h"
#include "wave.h"

namespace mag {

constexpr int CG_TPB = NC_MAX;  // one thread per cluster orbital
constexpr int CG_WAVES = CG_TPB / 64;
constexpr int CG_ENT = CLUSTER_MAX * BLOCKS_MAX;
constexpr int CG_RED = 3 * COCG_NZ;

__device__ __forceinline__ int cg_find(const int32_t* a, int n, int key) {
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

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double den = fma(b.x, b.x, b.y * b.y);
  return make_double2(fma(a.x, b.x, a.y * b.y) / den, fma(a.y, b.x, -a.x * b.y) / den);
}

// every thread receives the workgroup sums of its first K values
template <int K>
__device__ __forceinline__ void block_sums(double* v, double (*s_red)[CG_RED]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double t = wave_allreduce(v[k]);
    if (lane == 0) s_red[wave][k] = t;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = s_red[0][k];
  // waves in a fixed order, K values at a time (a full unroll would hold all
  // K x waves partial sums in registers at once)
#pragma unroll 1
  for (int w = 1; w < CG_WAVES; ++w) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += s_red[w][k];
  }
  __syncthreads();
}

__global__ __launch_bounds__(CG_TPB) void cocg_kernel(CocgArgs a) {
  __shared__ int32_t s_atoms[CLUSTER_MAX];
  __shared__ int32_t s_lptr[CLUSTER_MAX + 1];
  __shared__ uint16_t s_ent[CG_ENT];
  __shared__ double2 s_p[COCG_NZ][NC_MAX];
  __shared__ double s_red[CG_WAVES][CG_RED];
  __shared__ int s_flag;

  const int tid = threadIdx.x;
  const int64_t col = blockIdx.x;
  if (col >= a.ncols) return;
  const int j = a.cols[col];
  const int J = j >> 2, alpha = j & 3;
  const int64_t c0 = a.clus_ptr[J];
  const int nat = (int)(a.clus_ptr[J + 1] - c0);
  const int nC = NORB * nat;
  if (nat <= 0 || nat > CLUSTER_MAX) {
    if (tid == 0) atomicOr(a.err, (int)KERR_CAPACITY);
    return;
  }
  for (int i = tid; i < nat; i += CG_TPB) s_atoms[i] = a.clus_atoms[c0 + i];
  __syncthreads();

  // local block-CSR: one thread per cluster atom keeps the blocks of its
  // global row whose column atom is in the cluster
  int cnt = 0;
  if (tid < nat) {
    const int I = s_atoms[tid];
    for (int b = a.bptr[I]; b < a.bptr[I + 1]; ++b) cnt += cg_find(s_atoms, nat, a.bcol[b]) >= 0;
    s_lptr[tid + 1] = cnt;
  }
  if (tid == 0) s_lptr[0] = 0;
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < nat; ++i) s_lptr[i + 1] += s_lptr[i];
    s_flag = s_lptr[nat] > CG_ENT;
  }
  __syncthreads();
  if (s_flag) {
    if (tid == 0) atomicOr(a.err, (int)KERR_CAPACITY);
    return;
  }
  if (tid < nat) {
    const int I = s_atoms[tid];
    const int b0 = a.bptr[I];
    int e = s_lptr[tid];
    for (int b = b0; b < a.bptr[I + 1]; ++b) {
      const int kl = cg_find(s_atoms, nat, a.bcol[b]);
      if (kl >= 0) s_ent[e++] = (uint16_t)(((b - b0) << 8) | kl);
    }
  }
  const int jl = cg_find(s_atoms, nat, J);
  __syncthreads();
  if (jl < 0) {
    if (tid == 0) atomicOr(a.err, (int)KERR_PATTERN);
    return;
  }
  const int ell = NORB * jl + alpha;

  // this thread's row: its entry range and its place in the global blocks
  // (row a of a block: doubles 2a, 2a+1 of each 8-double quarter; S at +16)
  const int r = tid;
  const bool row = r < nC;
  int e0 = 0, e1 = 0;
  const double* rowp = a.bval;
  if (row) {
    e0 = s_lptr[r >> 2];
    e1 = s_lptr[(r >> 2) + 1];
    rowp = a.bval + (int64_t)a.bptr[s_atoms[r >> 2]] * 32 + 2 * (r & 3);
  }

  const int nq = min(COCG_NZ, a.nz - a.q0);
  double2 zq[COCG_NZ], x[COCG_NZ], res[COCG_NZ], p[COCG_NZ], rho[COCG_NZ];
  int state[COCG_NZ];  // 0 running, k > 0 converged after k steps, -1 failed, -2 unused
#pragma unroll
  for (int q = 0; q < COCG_NZ; ++q) {
    zq[q] = q < nq ? make_double2(a.z[2 * (a.q0 + q)], a.z[2 * (a.q0 + q) + 1])
                   : make_double2(0.0, 0.0);
    x[q] = make_double2(0.0, 0.0);
    res[q] = make_double2(r == ell ? 1.0 : 0.0, 0.0);
    p[q] = res[q];
    rho[q] = make_double2(1.0, 0.0);  // <e_l, e_l>
    state[q] = q < nq ? 0 : -2;
  }

  for (int it = 0; it < a.max_iter; ++it) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < COCG_NZ; ++q) any |= state[q] == 0;
    if (!any) break;
    if (row) {
#pragma unroll
      for (int q = 0; q < COCG_NZ; ++q) s_p[q][r] = p[q];
    }
    __syncthreads();
    // v = z S_C p - H_C p, the H and S blocks read once for all energies
    double2 hp[COCG_NZ], sp[COCG_NZ];
#pragma unroll
    for (int q = 0; q < COCG_NZ; ++q) {
      hp[q] = make_double2(0.0, 0.0);
      sp[q] = make_double2(0.0, 0.0);
    }
#pragma unroll 1
    for (int e = e0; e < e1; ++e) {
      const unsigned pe = s_ent[e];
      const double* bl = rowp + (pe >> 8) * 32;
      const double2 h01 = *reinterpret_cast<const double2*>(bl);
      const double2 h23 = *reinterpret_cast<const double2*>(bl + 8);
      const double2 s01 = *reinterpret_cast<const double2*>(bl + 16);
      const double2 s23 = *reinterpret_cast<const double2*>(bl + 24);
      const int k0 = NORB * (int)(pe & 255);
#pragma unroll
      for (int q = 0; q < COCG_NZ; ++q) {
        const double2 p0 = s_p[q][k0], p1 = s_p[q][k0 + 1], p2 = s_p[q][k0 + 2],
                      p3 = s_p[q][k0 + 3];
        hp[q].x = fma(h01.x, p0.x, fma(h01.y, p1.x, fma(h23.x, p2.x, fma(h23.y, p3.x, hp[q].x))));
        hp[q].y = fma(h01.x, p0.y, fma(h01.y, p1.y, fma(h23.x, p2.y, fma(h23.y, p3.y, hp[q].y))));
        sp[q].x = fma(s01.x, p0.x, fma(s01.y, p1.x, fma(s23.x, p2.x, fma(s23.y, p3.x, sp[q].x))));
        sp[q].y = fma(s01.x, p0.y, fma(s01.y, p1.y, fma(s23.x, p2.y, fma(s23.y, p3.y, sp[q].y))));
      }
    }
    double red[CG_RED];
#pragma unroll
    for (int q = 0; q < COCG_NZ; ++q) {
      const double2 zs = cmul(zq[q], sp[q]);
      hp[q] = make_double2(zs.x - hp[q].x, zs.y - hp[q].y);  // v
      const double2 d = cmul(p[q], hp[q]);
      red[2 * q] = d.x;
      red[2 * q + 1] = d.y;
    }
    block_sums<2 * COCG_NZ>(red, s_red);
#pragma unroll
    for (int q = 0; q < COCG_NZ; ++q) {
      if (state[q] != 0) continue;
      const double2 d = make_double2(red[2 * q], red[2 * q + 1]);
      if (!(d.x != 0.0 || d.y != 0.0) || !isfinite(d.x) || !isfinite(d.y)) {
        state[q] = -1;  // breakdown: <p, A p> = 0
        continue;
      }
      const double2 al = cdiv(rho[q], d);
      x[q] = make_double2(fma(al.x, p[q].x, fma(-al.y, p[q].y, x[q].x)),
                          fma(al.x, p[q].y, fma(al.y, p[q].x, x[q].y)));
      res[q] = make_double2(fma(-al.x, hp[q].x, fma(al.y, hp[q].y, res[q].x)),
                            fma(-al.x, hp[q].y, fma(-al.y, hp[q].x, res[q].y)));
    }
#pragma unroll
    for (int q = 0; q < COCG_NZ; ++q) {
      const double2 rr = cmul(res[q], res[q]);
      red[3 * q] = rr.x;
      red[3 * q + 1] = rr.y;
      red[3 * q + 2] = fma(res[q].x, res[q].x, res[q].y * res[q].y);
    }
    block_sums<3 * COCG_NZ>(red, s_red);
#pragma unroll
    for (int q = 0; q < COCG_NZ; ++q) {
      if (state[q] != 0) continue;
      if (!isfinite(red[3 * q + 2])) {
        state[q] = -1;
        continue;
      }
      if (sqrt(red[3 * q + 2]) <= a.tol) {  // |b| = 1
        state[q] = it + 1;
        continue;
      }
      const double2 rn = make_double2(red[3 * q], red[3 * q + 1]);
      if (!(rn.x != 0.0 || rn.y != 0.0)) {
        state[q] = -1;  // breakdown: <r, r> = 0 with r != 0
        continue;
      }
      const double2 beta = cdiv(rn, rho[q]);
      rho[q] = rn;
      const double2 bp = cmul(beta, p[q]);
      p[q] = make_double2(res[q].x + bp.x, res[q].y + bp.y);
    }
  }

  // static indices only (a runtime bound on q would move the arrays to scratch)
#pragma unroll
  for (int q = 0; q < COCG_NZ; ++q) {
    if (q < nq) {
      if (row) {
        double* g = a.G + 2 * (a.off[col] * (int64_t)a.nz + (int64_t)(a.q0 + q) * nC + r);
        g[0] = x[q].x;
        g[1] = x[q].y;
      }
      if (tid == 0) a.iters[col * a.nz + a.q0 + q] = state[q] > 0 ? state[q] : -1;
    }
  }
}

hipError_t launch_cocg(const CocgArgs& a, hipStream_t s) {
  if (a.ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(cocg_kernel, dim3((unsigned)a.ncols), dim3(CG_TPB), 0, s, a);
  return hipGetLastError();
}

}  // namespace mag
