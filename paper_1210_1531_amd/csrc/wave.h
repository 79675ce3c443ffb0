// Deterministic wave-level reductions of FP64 values on gfx950.
//
// The two cross-row levels use v_permlane32_swap / v_permlane16_swap, which
// exchange halves of two registers between lane groups, so a reduce-scatter
// step needs no per-lane selects; the four levels inside a row of 16 lanes use
// DPP moves (row_mirror, row_half_mirror, quad xor 2, quad xor 1), which pair
// lanes i with 15-i, then mirror within 8, then i^2, then i^1 -- a valid
// butterfly over the 16 lanes.  The summation order is fixed, so results are
// bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

namespace mag {

constexpr int DPP_ROW_MIRROR = 0x140;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_QUAD_XOR1 = 0xB1;  // quad_perm [1,0,3,2]

// DPP move of a double: every lane is written, so no old value is needed
// (a tied old operand would cost a register copy per use)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// DPP move writing only the lanes of the enabled banks; the others are left
// undefined (callers overwrite them)
template <int CTRL, int BANKS>
__device__ __forceinline__ double dpp_part(double src) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(src), CTRL, 0xF, BANKS, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(src), CTRL, 0xF, BANKS, false);
  return __hiloint2double(hi, lo);
}

// sum over the 16 lanes of each row; every lane of the row gets the total
__device__ __forceinline__ double row_allreduce(double x) {
  x += dpp_f64<DPP_ROW_MIRROR>(x);
  x += dpp_f64<DPP_ROW_HALF_MIRROR>(x);
  x += dpp_f64<DPP_QUAD_XOR2>(x);
  x += dpp_f64<DPP_QUAD_XOR1>(x);
  return x;
}

// a in lanes 0-31 keeps a, lanes 32-63 receive b of the partner half:
// returns a(l) + a(l^32) in lanes 0-31 and b(l^32) + b(l) in lanes 32-63
__device__ __forceinline__ double swap32_add(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// rows 0 and 2 (lane bit 4 clear) get a(l) + a(l^16), rows 1 and 3 get b(l^16) + b(l)
__device__ __forceinline__ double swap16_add(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// total over all 64 lanes, in every lane
__device__ __forceinline__ double wave_allreduce(double x) {
  x = swap32_add(x, x);
  x = swap16_add(x, x);
  return row_allreduce(x);
}

// DPP move with a bank mask: lanes of the enabled banks (groups of four lanes
// in a row) take src as permuted by CTRL, the other lanes keep old
template <int CTRL, int BANKS>
__device__ __forceinline__ double dpp_bank(double old, double src) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(src), CTRL, 0xF,
                                             BANKS, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(src), CTRL, 0xF,
                                             BANKS, false);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_IDENTITY = 0xE4;  // quad_perm [0,1,2,3]
constexpr int BANKS_B3 = 0xC;       // lanes with bit 3 set (banks 2, 3 of a row)
constexpr int BANKS_NB3 = 0x3;
constexpr int BANKS_B2 = 0xA;       // lanes with bit 2 set (banks 1, 3)
constexpr int BANKS_NB2 = 0x5;

// reduce-scatter of the pair (a, b) between lane i and its row mirror 15 - i
// (which differs in bit 3): lanes with bit 3 clear return a(i) + a(15-i), the
// others b(i) + b(15-i)
__device__ __forceinline__ double rs_mirror(double a, double b) {
  double recv = dpp_part<DPP_ROW_MIRROR, BANKS_NB3>(a);
  recv = dpp_bank<DPP_ROW_MIRROR, BANKS_B3>(recv, b);
  const double keep = dpp_bank<DPP_IDENTITY, BANKS_B3>(a, b);
  return keep + recv;
}
// the same between lane i and its half-row mirror (differs in bit 2)
__device__ __forceinline__ double rs_half_mirror(double a, double b) {
  double recv = dpp_part<DPP_ROW_HALF_MIRROR, BANKS_NB2>(a);
  recv = dpp_bank<DPP_ROW_HALF_MIRROR, BANKS_B2>(recv, b);
  const double keep = dpp_bank<DPP_IDENTITY, BANKS_B2>(a, b);
  return keep + recv;
}

// 16 values per lane -> the return value is the wave total of value
// 8 b5 + 4 b4 + 2 b2 + b3 (b_n: bit n of the lane id), the same in each quad
__device__ __forceinline__ double reduce16(double* v) {
#pragma unroll
  for (int t = 0; t < 8; ++t) v[t] = swap32_add(v[t], v[t + 8]);
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = swap16_add(v[t], v[t + 4]);
  const double u0 = rs_mirror(v[0], v[1]);
  const double u1 = rs_mirror(v[2], v[3]);
  double r = rs_half_mirror(u0, u1);
  r += dpp_f64<DPP_QUAD_XOR2>(r);
  r += dpp_f64<DPP_QUAD_XOR1>(r);
  return r;
}

// 8 values per lane -> the wave total of value 4 b5 + 2 b4 + b3, the same in
// each group of eight lanes
__device__ __forceinline__ double reduce8(double* v) {
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = swap32_add(v[t], v[t + 4]);
#pragma unroll
  for (int t = 0; t < 2; ++t) v[t] = swap16_add(v[t], v[t + 2]);
  double r = rs_mirror(v[0], v[1]);
  r += dpp_f64<DPP_ROW_HALF_MIRROR>(r);
  r += dpp_f64<DPP_QUAD_XOR2>(r);
  r += dpp_f64<DPP_QUAD_XOR1>(r);
  return r;
}

// 32 values per lane -> v[t], t < 8, holds the total of value 16 * b5 + 8 * b4 + t
__device__ __forceinline__ void reduce32(double* v) {
#pragma unroll
  for (int t = 0; t < 16; ++t) v[t] = swap32_add(v[t], v[t + 16]);
#pragma unroll
  for (int t = 0; t < 8; ++t) v[t] = swap16_add(v[t], v[t + 8]);
#pragma unroll
  for (int t = 0; t < 8; ++t) v[t] = row_allreduce(v[t]);
}

// 4 values per lane -> v[0] holds the total of value 2 * b5 + b4
__device__ __forceinline__ void reduce4(double* v) {
#pragma unroll
  for (int t = 0; t < 2; ++t) v[t] = swap32_add(v[t], v[t + 2]);
  v[0] = swap16_add(v[0], v[1]);
  v[0] = row_allreduce(v[0]);
}

}  // namespace mag
