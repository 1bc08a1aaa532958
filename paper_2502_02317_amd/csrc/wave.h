// Wavefront (64-lane) reductions on gfx950 through DPP lane moves, which stay
// in the VALU instead of round-tripping through LDS like a permute shuffle.
// All 64 lanes must be active where these are called.
#pragma once

#include <hip/hip_runtime.h>

namespace spg {

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane63(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum over the wave, returned to every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);        // row_ror:4
  v += dpp_move<0x128>(v);        // row_ror:8  -> every lane holds its row sum
  v += dpp_move<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3 -> lane 63 = total
  return lane63(v);
}

// Sum over each row of 16 lanes, returned to every lane of that row (all 16
// lanes of the row must be active).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);        // row_ror:4
  v += dpp_move<0x128>(v);        // row_ror:8
  return v;
}

// Sums of four values over the wave.  On return row r (lanes 16r..16r+15)
// holds the total of v_r in every lane (read it with a readlane of lane 16r).
// A swap between the wave's halves (v0,v2) and (v1,v3), then one between its
// rows, leave row r with partial sums of v_r alone, so the four totals share
// one 16-lane DPP sum: 21 instructions instead of four full reductions.
__device__ __forceinline__ void swap_halves(double &x, double &y) {
  // x's lanes 32..63 <-> y's lanes 0..31
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x),
                                                   (unsigned)__double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x),
                                                   (unsigned)__double2hiint(y), false, false);
  x = __hiloint2double((int)hi[0], (int)lo[0]);
  y = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void swap_rows(double &x, double &y) {
  // x's odd rows <-> y's even rows
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x),
                                                   (unsigned)__double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x),
                                                   (unsigned)__double2hiint(y), false, false);
  x = __hiloint2double((int)hi[0], (int)lo[0]);
  y = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double wave_sum4(double v0, double v1, double v2, double v3) {
  swap_halves(v0, v2);          // lanes 0..31: own v0 / partner's v0; 32..63: v2 likewise
  swap_halves(v1, v3);
  double a = v0 + v2;           // v0 partials in lanes 0..31, v2 partials in 32..63
  double b = v1 + v3;           // v1 partials in lanes 0..31, v3 partials in 32..63
  swap_rows(a, b);              // rows 0..3 of a: v0, v1, v2, v3 partials; b likewise
  return row16_sum(a + b);
}

// Max over the wave, returned to every lane (max(x, 0-fill) is safe for the
// non-negative arguments it is used with).
__device__ __forceinline__ double wave_max_nonneg(double v) {
  v = fmax(v, dpp_move<0xB1>(v));
  v = fmax(v, dpp_move<0x4E>(v));
  v = fmax(v, dpp_move<0x124>(v));
  v = fmax(v, dpp_move<0x128>(v));
  v = fmax(v, dpp_move<0x142, 0xA>(v));
  v = fmax(v, dpp_move<0x143, 0xC>(v));
  return lane63(v);
}

}  // namespace spg
