// Layout conversion of the caller's CSR into 4x4 atom blocks, checks and
// small fill kernels.
#include "mag_internal.h"

namespace mag {

static unsigned nblocks(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

// Verify the block-complete layout of row block J and record its block columns.
__global__ void check_layout_kernel(const int64_t* rowptr, const int32_t* colind, int64_t n,
                                    const int32_t* bptr, int32_t* bcol, int32_t* err) {
  const int64_t J = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (J >= n) return;
  const int nb = bptr[J + 1] - bptr[J];
  const int64_t r0 = rowptr[NORB * J];
  bool ok = nb >= 1;
  bool self = false;
  int prev = -1;
  for (int t = 0; t < nb && ok; ++t) {
    const int c0 = colind[r0 + 4 * t];
    if (c0 < 0 || (c0 & 3) != 0 || c0 / 4 >= n) {
      ok = false;
      break;
    }
    const int K = c0 >> 2;
    if (K <= prev) ok = false;
    prev = K;
    if (K == J) self = true;
    for (int a = 0; a < NORB && ok; ++a) {
      const int64_t ra = rowptr[NORB * J + a] + 4 * t;
      for (int be = 0; be < NORB; ++be)
        if (colind[ra + be] != NORB * K + be) ok = false;
    }
    bcol[bptr[J] + t] = K;
  }
  if (!ok || !self) atomicOr(err, (int)KERR_LAYOUT);
}

// one thread per value of the block layout: atom J, its block t (< 32) and
// the value o of the block's 32 (quarters of 8 doubles: H columns 0-1, H
// columns 2-3, S columns 0-1, S columns 2-3, each holding rows 0..3 as
// pairs, so that the four threads of an atom row in the Krylov SpMV read one
// contiguous 64-byte run per 16-byte load); a block's 32 stores are
// consecutive
__global__ void to_blocks_kernel(const int64_t* rowptr, const double* H, const double* S,
                                 int64_t n, const int32_t* bptr, double* bval) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t J = idx >> 10;
  if (J >= n) return;
  const int t = (int)((idx >> 5) & 31), o = (int)(idx & 31);
  if (t >= bptr[J + 1] - bptr[J]) return;
  const int q = o & 15, r = q & 7;
  const int a = r >> 1, be = (q >> 3) * 2 + (r & 1);
  const double* src = (o < 16) ? H : S;
  bval[(int64_t)(bptr[J] + t) * 32 + o] = src[rowptr[NORB * J + a] + 4 * t + be];
}

// one thread per block (atom J, block t < 32): the position of block (K, J)
// in row K, by binary search
__global__ void block_transpose_kernel(const int32_t* bptr, const int32_t* bcol, int64_t n,
                                       int32_t* btrans, int32_t* err) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t J = idx >> 5;
  if (J >= n) return;
  const int t = (int)(idx & 31);
  if (t >= bptr[J + 1] - bptr[J]) return;
  const int b = bptr[J] + t;
  const int K = bcol[b];
  int lo = bptr[K], hi = bptr[K + 1] - 1, found = -1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = bcol[mid];
    if (v == (int)J) {
      found = mid;
      break;
    }
    if (v < (int)J) lo = mid + 1;
    else hi = mid - 1;
  }
  btrans[b] = found;
  if (found < 0) atomicOr(err, (int)KERR_LAYOUT);
}

__global__ void check_finite_kernel(const double* x, int64_t n, int32_t* err) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) bad = true;
  if (bad) atomicOr(err, (int)KERR_NONFINITE);
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void scale_copy_kernel(const double* x, int64_t n, double a, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

static unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_check_layout(const int64_t* rowptr, const int32_t* colind, int64_t n,
                               const int32_t* bptr, int32_t* bcol, int32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(check_layout_kernel, dim3(nblocks(n, 128)), dim3(128), 0, s, rowptr, colind,
                     n, bptr, bcol, err);
  return hipGetLastError();
}
hipError_t launch_to_blocks(const int64_t* rowptr, const double* H, const double* S, int64_t n,
                            const int32_t* bptr, double* bval, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_blocks_kernel, dim3(nblocks(n * 1024, 256)), dim3(256), 0, s, rowptr, H, S, n,
                     bptr, bval);
  return hipGetLastError();
}
hipError_t launch_block_transpose(const int32_t* bptr, const int32_t* bcol, int64_t n,
                                  int32_t* btrans, int32_t* err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(block_transpose_kernel, dim3(nblocks(n * 32, 256)), dim3(256), 0, s, bptr, bcol,
                     n, btrans, err);
  return hipGetLastError();
}
hipError_t launch_check_finite(const double* x, int64_t n, int32_t* err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, err);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_scale_copy(const double* x, int64_t n, double a, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_copy_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, a, y);
  return hipGetLastError();
}

}  // namespace mag

namespace mag {

// nonzeros of H_C (16 per block with both atoms in the cluster), per atom
__global__ void cluster_nnz_kernel(const int32_t* bptr, const int32_t* bcol,
                                   const int64_t* clus_ptr, const int32_t* clus_atoms, int64_t n,
                                   int64_t* out) {
  const int64_t J = blockIdx.x;
  if (J >= n) return;
  const int64_t c0 = clus_ptr[J];
  const int nat = (int)(clus_ptr[J + 1] - c0);
  int64_t cnt = 0;
  for (int i = threadIdx.x; i < nat; i += blockDim.x) {
    const int I = clus_atoms[c0 + i];
    for (int b = bptr[I]; b < bptr[I + 1]; ++b) {
      const int K = bcol[b];
      int lo = 0, hi = nat - 1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = clus_atoms[c0 + mid];
        if (v == K) {
          cnt += 16;
          break;
        }
        if (v < K) lo = mid + 1;
        else hi = mid - 1;
      }
    }
  }
  for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
  __shared__ int64_t s_c[4];
  if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) out[J] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
}

hipError_t launch_cluster_nnz(const int32_t* bptr, const int32_t* bcol, const int64_t* clus_ptr,
                              const int32_t* clus_atoms, int64_t n, int64_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cluster_nnz_kernel, dim3((unsigned)n), dim3(256), 0, s, bptr, bcol, clus_ptr,
                     clus_atoms, n, out);
  return hipGetLastError();
}

}  // namespace mag
