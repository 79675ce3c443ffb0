// Tight-binding matrices from positions (two-center Slater-Koster sp model),
// their vector-Jacobian product (forces through the density matrix), the cell
// list shared with the cluster builder, and the cluster lists themselves.
//
// The letter builds H and S redundantly on every node instead of exchanging
// them; here they are built once on the device by one thread per block row.
#include <algorithm>

#include "mag_internal.h"
#include "sk_dev.h"

namespace mag {

constexpr int STPB = 128;

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
struct CellView {
  int nc[3];
  int brute;
  const int32_t* start;
  const int32_t* atoms;
};

__device__ __forceinline__ int cell_coord(double x, double L, int nc) {
  double f = x - L * floor(x / L);
  int c = (int)(f / L * nc);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

template <typename F>
__device__ __forceinline__ void for_candidates(const CellView& cv, const double* pos, int64_t n,
                                               const Box& box, int64_t i, F&& f) {
  if (cv.brute) {
    for (int64_t k = 0; k < n; ++k) f((int)k);
    return;
  }
  const int cx = cell_coord(pos[3 * i], box.L[0], cv.nc[0]);
  const int cy = cell_coord(pos[3 * i + 1], box.L[1], cv.nc[1]);
  const int cz = cell_coord(pos[3 * i + 2], box.L[2], cv.nc[2]);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = (cx + dx + cv.nc[0]) % cv.nc[0];
        const int y = (cy + dy + cv.nc[1]) % cv.nc[1];
        const int z = (cz + dz + cv.nc[2]) % cv.nc[2];
        const int c = (z * cv.nc[1] + y) * cv.nc[0] + x;
        for (int a = cv.start[c]; a < cv.start[c + 1]; ++a) f(cv.atoms[a]);
      }
}

__global__ void cell_assign_kernel(const double* pos, int64_t n, Box box, int nc0, int nc1,
                                   int nc2, int32_t* cell_of, int32_t* count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = cell_coord(pos[3 * i], box.L[0], nc0);
  const int y = cell_coord(pos[3 * i + 1], box.L[1], nc1);
  const int z = cell_coord(pos[3 * i + 2], box.L[2], nc2);
  const int c = (z * nc1 + y) * nc0 + x;
  cell_of[i] = c;
  atomicAdd(&count[c], 1);
}

__global__ void cell_fill_kernel(const int32_t* cell_of, int64_t n, const int32_t* start,
                                 int32_t* fillpos, int32_t* atoms) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cell_of[i];
  const int slot = atomicAdd(&fillpos[c], 1);
  atoms[start[c] + slot] = (int)i;
}

static unsigned blocks_for(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

hipError_t build_cell_list(CellList& cl, const double* pos, int64_t n, const double cell[3],
                           double rmin, hipStream_t s) {
  cl.brute = false;
  for (int d = 0; d < 3; ++d) {
    cl.ncell[d] = (int)std::floor(cell[d] / rmin);
    if (cl.ncell[d] < 3) cl.brute = true;
  }
  if (cl.brute || n == 0) {
    cl.brute = true;
    return hipSuccess;
  }
  const int64_t ncells = (int64_t)cl.ncell[0] * cl.ncell[1] * cl.ncell[2];
  hipError_t e;
  if ((e = cl.cell_of.reserve(n * 4)) != hipSuccess) return e;
  if ((e = cl.cell_count.reserve((ncells + 1) * 4)) != hipSuccess) return e;
  if ((e = cl.cell_start.reserve((ncells + 1) * 4)) != hipSuccess) return e;
  if ((e = cl.cell_atoms.reserve(n * 4)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(cl.cell_count.p, 0, (ncells + 1) * 4, s)) != hipSuccess) return e;
  Box box{{cell[0], cell[1], cell[2]}};
  hipLaunchKernelGGL(cell_assign_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos, n, box,
                     cl.ncell[0], cl.ncell[1], cl.ncell[2], cl.cell_of.as<int32_t>(),
                     cl.cell_count.as<int32_t>());
  std::vector<int32_t> cnt(ncells), start(ncells + 1);
  if ((e = hipMemcpyAsync(cnt.data(), cl.cell_count.p, ncells * 4, hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  start[0] = 0;
  for (int64_t c = 0; c < ncells; ++c) start[c + 1] = start[c] + cnt[c];
  if ((e = hipMemcpyAsync(cl.cell_start.p, start.data(), (ncells + 1) * 4, hipMemcpyHostToDevice,
                          s)) != hipSuccess)
    return e;
  if ((e = hipMemsetAsync(cl.cell_count.p, 0, (ncells + 1) * 4, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(cell_fill_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                     cl.cell_of.as<int32_t>(), n, cl.cell_start.as<int32_t>(),
                     cl.cell_count.as<int32_t>(), cl.cell_atoms.as<int32_t>());
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);  // keep the host vectors alive until the copies are done
}

static CellView view_of(const CellList& cl) {
  CellView v;
  v.nc[0] = cl.ncell[0];
  v.nc[1] = cl.ncell[1];
  v.nc[2] = cl.ncell[2];
  v.brute = cl.brute ? 1 : 0;
  v.start = cl.cell_start.as<int32_t>();
  v.atoms = cl.cell_atoms.as<int32_t>();
  return v;
}

// ---------------------------------------------------------------------------
// sparsity pattern: atoms closer than r_cut, plus self
// ---------------------------------------------------------------------------
__global__ void sk_count_kernel(const double* pos, int64_t n, Box box, double rc2, CellView cv,
                                int32_t* cnt, int32_t* err) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  int c = 1;
  for_candidates(cv, pos, n, box, i, [&](int k) {
    if (k == i) return;
    double dx = pos[3 * k] - xi, dy = pos[3 * k + 1] - yi, dz = pos[3 * k + 2] - zi;
    min_image(box, dx, dy, dz);
    if (dx * dx + dy * dy + dz * dz < rc2) ++c;
  });
  cnt[i] = c;
  if (c > BLOCKS_MAX) atomicOr(err, (int)KERR_CAPACITY);
}

__global__ void sk_fill_kernel(const double* pos, int64_t n, Box box, double rc2, CellView cv,
                               const int32_t* bptr, int32_t* bcol) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  int list[BLOCKS_MAX];
  int c = 0;
  list[c++] = (int)i;
  for_candidates(cv, pos, n, box, i, [&](int k) {
    if (k == i) return;
    double dx = pos[3 * k] - xi, dy = pos[3 * k + 1] - yi, dz = pos[3 * k + 2] - zi;
    min_image(box, dx, dy, dz);
    if (dx * dx + dy * dy + dz * dz < rc2 && c < BLOCKS_MAX) list[c++] = k;
  });
  for (int a = 1; a < c; ++a) {  // insertion sort, ascending atom id
    const int v = list[a];
    int b = a - 1;
    while (b >= 0 && list[b] > v) {
      list[b + 1] = list[b];
      --b;
    }
    list[b + 1] = v;
  }
  const int base = bptr[i];
  for (int a = 0; a < c; ++a) bcol[base + a] = list[a];
}

__global__ void sk_csr_kernel(const int32_t* bptr, const int32_t* bcol, int64_t n,
                              int64_t* rowptr, int32_t* colind) {
  const int64_t J = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (J >= n) return;
  const int64_t b0 = bptr[J];
  const int nb = bptr[J + 1] - bptr[J];
  for (int a = 0; a < NORB; ++a) {
    const int64_t r0 = 16 * b0 + 4 * (int64_t)a * nb;
    rowptr[NORB * J + a] = r0;
    for (int t = 0; t < nb; ++t)
      for (int be = 0; be < NORB; ++be) colind[r0 + 4 * t + be] = NORB * bcol[b0 + t] + be;
  }
  if (J == n - 1) rowptr[NORB * n] = 16 * (int64_t)bptr[n];
}

// the same block split by bond type: sigma (V_ss, V_sp, V_pp sigma terms)
// and pi (the V_pp pi term of the p-p sub-block); Bs + Bp is two_center's block
__device__ __forceinline__ void two_center_split(const SKModelDev& m, const double* V, double dx,
                                                 double dy, double dz, double Bs[4][4],
                                                 double Bp[4][4]) {
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double l[3] = {dx / r, dy / r, dz / r};
  double u, du;
  radial(m, r, u, du);
  Bs[0][0] = V[0] * u;
  Bp[0][0] = 0.0;
  for (int a = 0; a < 3; ++a) {
    Bs[0][1 + a] = l[a] * V[1] * u;
    Bs[1 + a][0] = -l[a] * V[1] * u;
    Bp[0][1 + a] = 0.0;
    Bp[1 + a][0] = 0.0;
    for (int b = 0; b < 3; ++b) {
      const double ll = l[a] * l[b];
      Bs[1 + a][1 + b] = ll * V[2] * u;
      Bp[1 + a][1 + b] = ((a == b ? 1.0 : 0.0) - ll) * V[3] * u;
    }
  }
}

// integrated crystal orbital Hamiltonian populations per block of the pattern:
// block t of block row J (column atom K) gives B = sum_ab H_{Ja;Kb} rho_{Kb;Ja}
// from the system's H (block values) and rho (CSR layout of H), and its sigma
// and pi parts from the split SK block at the positions (zero on the diagonal).
// One thread per block; its row J by binary search in the block-row pointers.
__global__ void icohp_kernel(SKModelDev m, const double* pos, int64_t n, int64_t nblk, Box box,
                             const int32_t* bptr, const int32_t* bcol, const double* bval,
                             const double* rho, double* B, double* Bsig, double* Bpi) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  int64_t lo = 0, hi = n - 1;  // last row J with bptr[J] <= b
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (bptr[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const int64_t J = lo;
  const int64_t b0 = bptr[J];
  const int nb = bptr[J + 1] - bptr[J];
  const int t = (int)(b - b0);
  const int K = bcol[b];
  const double* hv = bval + b * 32;  // H: quarters of row pairs (see to_blocks)
  double rb[4][4];
  double full = 0.0;
  for (int a = 0; a < 4; ++a) {
    const double2* rr = reinterpret_cast<const double2*>(rho + 16 * b0 + 4 * (int64_t)a * nb + 4 * t);
    const double2 r01 = rr[0], r23 = rr[1];
    rb[a][0] = r01.x;
    rb[a][1] = r01.y;
    rb[a][2] = r23.x;
    rb[a][3] = r23.y;
    for (int c = 0; c < 4; ++c) full = fma(hv[(c >> 1) * 8 + 2 * a + (c & 1)], rb[a][c], full);
  }
  double sig = 0.0, pi = 0.0;
  if (K != J) {
    double dx = pos[3 * K] - pos[3 * J], dy = pos[3 * K + 1] - pos[3 * J + 1],
           dz = pos[3 * K + 2] - pos[3 * J + 2];
    min_image(box, dx, dy, dz);
    double Bs[4][4], Bp[4][4];
    two_center_split(m, m.vh, dx, dy, dz, Bs, Bp);
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) {
        sig = fma(Bs[a][c], rb[a][c], sig);
        pi = fma(Bp[a][c], rb[a][c], pi);
      }
  }
  if (B) B[b] = full;
  if (Bsig) Bsig[b] = sig;
  if (Bpi) Bpi[b] = pi;
}

// one thread per block (atom J, block t < 32 of its row)
__global__ void sk_values_kernel(SKModelDev m, const double* pos, int64_t n, Box box,
                                 const int32_t* bptr, const int32_t* bcol, double* H, double* S) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t J = idx >> 5;
  if (J >= n) return;
  const int t = (int)(idx & 31);
  const int64_t b0 = bptr[J];
  const int nb = bptr[J + 1] - bptr[J];
  if (t >= nb) return;
  const int K = bcol[b0 + t];
  double Bh[4][4], Bs[4][4];
  if (K == J) {
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) {
        Bh[a][c] = (a == c) ? (a == 0 ? m.es : m.ep) : 0.0;
        Bs[a][c] = (a == c) ? 1.0 : 0.0;
      }
  } else {
    double dx = pos[3 * K] - pos[3 * J], dy = pos[3 * K + 1] - pos[3 * J + 1],
           dz = pos[3 * K + 2] - pos[3 * J + 2];
    min_image(box, dx, dy, dz);
    two_center(m, m.vh, dx, dy, dz, Bh);
    two_center(m, m.vs, dx, dy, dz, Bs);
  }
  for (int a = 0; a < 4; ++a) {
    const int64_t r0 = 16 * b0 + 4 * (int64_t)a * nb + 4 * t;
    for (int c = 0; c < 4; ++c) {
      H[r0 + c] = Bh[a][c];
      S[r0 + c] = Bs[a][c];
    }
  }
}

// grad[I] = sum over blocks (I,K) and (K,I) of g . d(block)/dR_I, in two
// passes: one thread per block b = (I, t) of the pattern writes the pair's
// two terms (block (I,K) and its transpose (K,I) in row K) to part[b], then
// one thread per atom adds its row's parts in block order (deterministic).
// One thread per atom alone would leave most of the device idle: its ~17
// blocks x 4 contractions run as one serial chain per thread.
__global__ void sk_vjp_pair_kernel(SKModelDev m, const double* pos, int64_t n, int64_t nblk,
                                   Box box, const int32_t* bptr, const int32_t* bcol,
                                   const int32_t* btrans, const double* gH, const double* gS,
                                   double sgn, double* part) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  int64_t lo = 0, hi = n - 1;  // last row I with bptr[I] <= b
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (bptr[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const int64_t I = lo;
  const int64_t b0 = bptr[I];
  const int nb = bptr[I + 1] - bptr[I];
  const int t = (int)(b - b0);
  const int K = bcol[b];
  double acc[3] = {0.0, 0.0, 0.0};
  if (K != I) {
    double dx = pos[3 * K] - pos[3 * I], dy = pos[3 * K + 1] - pos[3 * I + 1],
           dz = pos[3 * K + 2] - pos[3 * I + 2];
    min_image(box, dx, dy, dz);
    // block (I, K): depends on R_I through d = R_K - R_I  -> minus sign
    {
      double Gh[4][4], Gs[4][4];
      for (int a = 0; a < 4; ++a) {
        const int64_t r0 = 16 * b0 + 4 * (int64_t)a * nb + 4 * t;
        for (int c = 0; c < 4; ++c) {
          Gh[a][c] = gH[r0 + c];
          Gs[a][c] = sgn * gS[r0 + c];
        }
      }
      double oh[3], os[3];
      two_center_contract(m, m.vh, dx, dy, dz, Gh, oh);
      two_center_contract(m, m.vs, dx, dy, dz, Gs, os);
      for (int c = 0; c < 3; ++c) acc[c] -= oh[c] + os[c];
    }
    // block (K, I) in row K: depends on R_I through d' = R_I - R_K = -d -> plus sign
    {
      const int bt = btrans[b];
      const int64_t k0 = bptr[K];
      const int nbk = bptr[K + 1] - bptr[K];
      const int tt = (int)(bt - k0);
      double Gh[4][4], Gs[4][4];
      for (int a = 0; a < 4; ++a) {
        const int64_t r0 = 16 * k0 + 4 * (int64_t)a * nbk + 4 * tt;
        for (int c = 0; c < 4; ++c) {
          Gh[a][c] = gH[r0 + c];
          Gs[a][c] = sgn * gS[r0 + c];
        }
      }
      double oh[3], os[3];
      two_center_contract(m, m.vh, -dx, -dy, -dz, Gh, oh);
      two_center_contract(m, m.vs, -dx, -dy, -dz, Gs, os);
      for (int c = 0; c < 3; ++c) acc[c] += oh[c] + os[c];
    }
  }
  for (int c = 0; c < 3; ++c) part[3 * b + c] = acc[c];
}

__global__ void sk_vjp_sum_kernel(const int32_t* bptr, int64_t n, const double* part,
                                  double* grad) {
  const int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (I >= n) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t b = bptr[I]; b < bptr[I + 1]; ++b)
    for (int c = 0; c < 3; ++c) acc[c] += part[3 * b + c];
  for (int c = 0; c < 3; ++c) grad[3 * I + c] = acc[c];
}

// Pair repulsion of the total energy: phi(r) = phi0 (r0 / r)^m fc(r) over
// the atom pairs of the pattern (one thread per atom J, its block row).  Both
// ends of a pair see it, so e[J] takes half of each phi; the force on J is
// sum_K phi'(r) d / r with d = R_K - R_J.
__global__ void pair_rep_kernel(SKModelDev m, const double* pos, int64_t n, Box box,
                                const int32_t* bptr, const int32_t* bcol, double phi0,
                                double mexp, double* e, double* F) {
  const int64_t J = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (J >= n) return;
  double eJ = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
  for (int64_t b = bptr[J]; b < bptr[J + 1]; ++b) {
    const int K = bcol[b];
    if (K == J) continue;
    double dx = pos[3 * K] - pos[3 * J], dy = pos[3 * K + 1] - pos[3 * J + 1],
           dz = pos[3 * K + 2] - pos[3 * J + 2];
    min_image(box, dx, dy, dz);
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(r < m.r_cut)) continue;
    double fc, dfc;
    smooth_cutoff(m, r, fc, dfc);
    const double g = phi0 * pow(m.r0 / r, mexp);
    const double dphi = (-mexp * g / r) * fc + g * dfc;
    eJ += 0.5 * (g * fc);
    const double c = dphi / r;
    fx += c * dx;
    fy += c * dy;
    fz += c * dz;
  }
  e[J] = eJ;
  F[3 * J] = fx;
  F[3 * J + 1] = fy;
  F[3 * J + 2] = fz;
}

hipError_t launch_pair_rep(const SKModelDev& m, const double* pos, int64_t n, const double cell[3],
                           const int32_t* bptr, const int32_t* bcol, double phi0, double mexp,
                           double* e, double* F, hipStream_t s) {
  Box box{{cell[0], cell[1], cell[2]}};
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(pair_rep_kernel, dim3(blocks_for(n, STPB)), dim3(STPB), 0, s, m, pos, n, box,
                     bptr, bcol, phi0, mexp, e, F);
  return hipGetLastError();
}

hipError_t launch_sk_count(const double* pos, int64_t n, const double cell[3], double rc,
                           const CellList& cl, int32_t* cnt, int32_t* err, hipStream_t s) {
  Box box{{cell[0], cell[1], cell[2]}};
  hipLaunchKernelGGL(sk_count_kernel, dim3(blocks_for(n, STPB)), dim3(STPB), 0, s, pos, n, box,
                     rc * rc, view_of(cl), cnt, err);
  return hipGetLastError();
}
hipError_t launch_sk_fill(const double* pos, int64_t n, const double cell[3], double rc,
                          const CellList& cl, const int32_t* bptr, int32_t* bcol, hipStream_t s) {
  Box box{{cell[0], cell[1], cell[2]}};
  hipLaunchKernelGGL(sk_fill_kernel, dim3(blocks_for(n, STPB)), dim3(STPB), 0, s, pos, n, box,
                     rc * rc, view_of(cl), bptr, bcol);
  return hipGetLastError();
}
hipError_t launch_sk_csr(const int32_t* bptr, const int32_t* bcol, int64_t n, int64_t* rowptr,
                         int32_t* colind, hipStream_t s) {
  hipLaunchKernelGGL(sk_csr_kernel, dim3(blocks_for(n, STPB)), dim3(STPB), 0, s, bptr, bcol, n,
                     rowptr, colind);
  return hipGetLastError();
}
hipError_t launch_sk_values(const SKModelDev& m, const double* pos, int64_t n,
                            const double cell[3], const int32_t* bptr, const int32_t* bcol,
                            double* H, double* S, hipStream_t s) {
  Box box{{cell[0], cell[1], cell[2]}};
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sk_values_kernel, dim3(blocks_for(n * 32, STPB)), dim3(STPB), 0, s, m, pos, n,
                     box, bptr, bcol, H, S);
  return hipGetLastError();
}
hipError_t launch_sk_vjp(const SKModelDev& m, const double* pos, int64_t n, int64_t nblk,
                         const double cell[3], const int32_t* bptr, const int32_t* bcol,
                         const int32_t* btrans, const double* gH, const double* gS, double sign_gS,
                         double* part, double* grad, hipStream_t s) {
  Box box{{cell[0], cell[1], cell[2]}};
  if (n <= 0) return hipSuccess;
  if (nblk > 0)
    hipLaunchKernelGGL(sk_vjp_pair_kernel, dim3(blocks_for(nblk, STPB)), dim3(STPB), 0, s, m, pos,
                       n, nblk, box, bptr, bcol, btrans, gH, gS, sign_gS, part);
  hipLaunchKernelGGL(sk_vjp_sum_kernel, dim3(blocks_for(n, STPB)), dim3(STPB), 0, s, bptr, n, part,
                     grad);
  return hipGetLastError();
}

hipError_t launch_icohp(const SKModelDev& m, const double* pos, int64_t n, int64_t nblk,
                        const double cell[3], const int32_t* bptr, const int32_t* bcol,
                        const double* bval, const double* rho, double* B, double* Bsig,
                        double* Bpi, hipStream_t s) {
  Box box{{cell[0], cell[1], cell[2]}};
  if (n <= 0 || nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(icohp_kernel, dim3(blocks_for(nblk, STPB)), dim3(STPB), 0, s, m, pos, n, nblk,
                     box, bptr, bcol, bval, rho, B, Bsig, Bpi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// clusters: atoms within r_c of each atom (inclusive), sorted by id
// ---------------------------------------------------------------------------
constexpr int CTPB = 256;
constexpr int CSORT = 256;  // sort width (>= CLUSTER_MAX)

__global__ __launch_bounds__(CTPB) void cluster_scan_kernel(const double* pos, int64_t n, Box box,
                                                            double rc2, CellView cv,
                                                            int32_t* tmp, int32_t* cnt,
                                                            int32_t* err) {
  __shared__ int32_t s_list[CSORT];
  __shared__ int s_n;
  const int64_t J = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid == 0) s_n = 0;
  __syncthreads();
  const double xj = pos[3 * J], yj = pos[3 * J + 1], zj = pos[3 * J + 2];
  auto test = [&](int k) {
    double dx = pos[3 * k] - xj, dy = pos[3 * k + 1] - yj, dz = pos[3 * k + 2] - zj;
    min_image(box, dx, dy, dz);
    if (dx * dx + dy * dy + dz * dz <= rc2) {
      const int slot = atomicAdd(&s_n, 1);
      if (slot < CSORT) s_list[slot] = k;
    }
  };
  if (cv.brute) {
    for (int64_t k = tid; k < n; k += CTPB) test((int)k);
  } else {
    const int cx = cell_coord(xj, box.L[0], cv.nc[0]);
    const int cy = cell_coord(yj, box.L[1], cv.nc[1]);
    const int cz = cell_coord(zj, box.L[2], cv.nc[2]);
    for (int q = 0; q < 27; ++q) {
      const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
      const int x = (cx + dx + cv.nc[0]) % cv.nc[0];
      const int y = (cy + dy + cv.nc[1]) % cv.nc[1];
      const int z = (cz + dz + cv.nc[2]) % cv.nc[2];
      const int c = (z * cv.nc[1] + y) * cv.nc[0] + x;
      for (int a = cv.start[c] + tid; a < cv.start[c + 1]; a += CTPB) test(cv.atoms[a]);
    }
  }
  __syncthreads();
  const int total = s_n;
  if (total > CLUSTER_MAX) {
    if (tid == 0) {
      atomicOr(err, (int)KERR_CAPACITY);
      cnt[J] = 0;
    }
    return;
  }
  for (int a = total + tid; a < CSORT; a += CTPB) s_list[a] = 0x7fffffff;
  __syncthreads();
  // bitonic sort of CSORT keys
  for (int k = 2; k <= CSORT; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = tid; i < CSORT; i += CTPB) {
        const int p = i ^ jj;
        if (p > i) {
          const int a = s_list[i], b = s_list[p];
          const bool asc = (i & k) == 0;
          if ((a > b) == asc) {
            s_list[i] = b;
            s_list[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int a = tid; a < total; a += CTPB) tmp[J * (int64_t)CLUSTER_MAX + a] = s_list[a];
  if (tid == 0) cnt[J] = total;
}

__global__ void cluster_compact_kernel(const int32_t* tmp, const int32_t* cnt, const int64_t* ptr,
                                       int64_t n, int32_t* atoms) {
  const int64_t J = blockIdx.x;
  if (J >= n) return;
  for (int a = threadIdx.x; a < cnt[J]; a += blockDim.x)
    atoms[ptr[J] + a] = tmp[J * (int64_t)CLUSTER_MAX + a];
}

hipError_t launch_cluster_scan_cv(const double* pos, int64_t n, const double cell[3], double rc,
                                  const CellList& cl, int32_t* tmp, int32_t* cnt, int32_t* err,
                                  hipStream_t s) {
  Box box{{cell[0], cell[1], cell[2]}};
  hipLaunchKernelGGL(cluster_scan_kernel, dim3((unsigned)n), dim3(CTPB), 0, s, pos, n, box,
                     rc * rc, view_of(cl), tmp, cnt, err);
  return hipGetLastError();
}

hipError_t launch_cluster_compact(const int32_t* tmp, const int32_t* cnt, const int64_t* ptr,
                                  int64_t n, int32_t* atoms, hipStream_t s) {
  hipLaunchKernelGGL(cluster_compact_kernel, dim3((unsigned)n), dim3(64), 0, s, tmp, cnt, ptr, n,
                     atoms);
  return hipGetLastError();
}

}  // namespace mag
