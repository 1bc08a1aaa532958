// Device helpers shared by the search kernels: site fields and energies,
// order-preserving keys, block scans, radix-select steps and a bitonic sort.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cstdint>

#include "spg_internal.h"

namespace spg {

// Class-batched launches: the instance's own tables.
__device__ __forceinline__ void shift_tabs(SearchTabs &t, long ist) {
  SPG_INST(t.E_loc);
  SPG_INST(t.E_h);
  SPG_INST(t.E_v);
  SPG_INST(t.E_d);
  SPG_INST(t.E_a);
  SPG_INST(t.W_v);
  SPG_INST(t.W_d);
  SPG_INST(t.W_a);
}

// g^b_c(s): couplings of x_{r,c} = s to the fixed row above (1 for r = 0).
__device__ __forceinline__ double field(const SearchTabs &t, int r, int c, const uint8_t *cb,
                                        int s) {
  if (r == 0) return 1.0;
  const int C = t.cols, d = t.d;
  const uint8_t *up = cb + (r - 1) * C;
  const long dd = (long)d * d;
  double g = t.W_v[((long)(r - 1) * C + c) * dd + up[c] * d + s];
  if (c > 0) g *= t.W_d[((long)(r - 1) * (C - 1) + (c - 1)) * dd + up[c - 1] * d + s];
  if (c < C - 1) g *= t.W_a[((long)(r - 1) * (C - 1) + c) * dd + up[c + 1] * d + s];
  return g;
}

// Energy added by x_{r,c} = s: the Eq. (1) terms that close at this site.
__device__ __forceinline__ double delta_energy(const SearchTabs &t, int r, int c,
                                               const uint8_t *cb, int s) {
  const int C = t.cols, d = t.d;
  const long dd = (long)d * d;
  double e = t.E_loc[((long)r * C + c) * d + s];
  if (c > 0) e += t.E_h[((long)r * (C - 1) + (c - 1)) * dd + cb[r * C + c - 1] * d + s];
  if (r > 0) {
    const uint8_t *up = cb + (r - 1) * C;
    e += t.E_v[((long)(r - 1) * C + c) * dd + up[c] * d + s];
    if (c > 0) e += t.E_d[((long)(r - 1) * (C - 1) + (c - 1)) * dd + up[c - 1] * d + s];
    if (c < C - 1) e += t.E_a[((long)(r - 1) * (C - 1) + c) * dd + up[c + 1] * d + s];
  }
  return e;
}

// A parent none of whose children has a positive conditional weight has no
// conditional from the contraction; it takes the conditional of the fixed
// sites' Boltzmann weight alone, p(s) = softmax_s(-beta dE(b, s)).  Every lane
// of the parent's wavefront calls this; it returns the normalisation of
// log p(s) = -beta (dE(s) - emin) - lse, reduced over the wavefront.
__device__ inline void local_softmax_norm(const SearchTabs &t, int r, int c, const uint8_t *cb,
                                          int lane, double &emin, double &lse) {
  double m = INFINITY;
  for (int s = lane; s < t.d; s += 64) m = fmin(m, delta_energy(t, r, c, cb, s));
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
  double z = 0.0;
  for (int s = lane; s < t.d; s += 64) z += exp(-t.beta * (delta_energy(t, r, c, cb, s) - m));
  for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o, 64);
  emin = m;
  lse = log(z);
}

// Key for ascending sort = descending score; NaN sorts with -inf.
__device__ __forceinline__ uint64_t desc_key(double v) {
  if (!(v == v)) v = -INFINITY;
  uint64_t u = __double_as_longlong(v);
  const uint64_t sign = 0x8000000000000000ull;
  u = (u & sign) ? ~u : (u | sign);   // ascending in v
  return ~u;                          // ascending in -v
}
__device__ __forceinline__ uint64_t asc_key(double v) {
  if (!(v == v)) v = INFINITY;
  uint64_t u = __double_as_longlong(v);
  const uint64_t sign = 0x8000000000000000ull;
  return (u & sign) ? ~u : (u | sign);
}

// Block-wide exclusive scan of 0/1 flags (blockDim = 1024); returns the prefix
// and writes the block total to *total.
__device__ inline int block_excl_scan(int f, int *wsum, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const unsigned long long mask = __ballot(f);
  const int pre = __popcll(mask & ((1ull << lane) - 1ull));
  __syncthreads();
  if (lane == 0) wsum[w] = __popcll(mask);
  __syncthreads();
  int off = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  *total = tot;
  return off + pre;
}

// Sort (key, id) pairs ascending with one workgroup (bitonic); the arrays may
// live in global memory or LDS (each call site is inlined with its own).
__device__ __forceinline__ void bitonic_sort(uint64_t *keys, int32_t *ids, int n_pow2) {
  for (int k = 2; k <= n_pow2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n_pow2; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t ki = keys[i], kj = keys[ixj];
          const int32_t ii = ids[i], ij = ids[ixj];
          const bool gt = (ki > kj) || (ki == kj && ii > ij);
          const bool up = ((i & k) == 0);
          if (gt == up) {
            keys[i] = kj; keys[ixj] = ki;
            ids[i] = ij; ids[ixj] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
}

// The same sort for (key, id) pairs held in LDS, blockDim = 1024, n_pow2 <=
// 8192: thread t keeps elements t + 1024 r in registers; stages whose partner
// lies in the same wavefront (distance < 64) exchange through lane shuffles
// without barriers, the others go through LDS.  Leaves the sorted pairs in LDS.
constexpr int kSortLdsRegs = 8;
__device__ inline void bitonic_sort_lds(uint64_t *keys, int32_t *ids, int n_pow2) {
  const int tid = threadIdx.x;
  const int R = (n_pow2 + 1023) >> 10;          // 1..kSortLdsRegs
  uint64_t kv[kSortLdsRegs];
  int32_t iv[kSortLdsRegs];
#pragma unroll
  for (int r = 0; r < kSortLdsRegs; ++r) {
    const int i = tid + 1024 * r;
    kv[r] = (r < R && i < n_pow2) ? keys[i] : ~0ull;
    iv[r] = (r < R && i < n_pow2) ? ids[i] : INT_MAX;
  }
  for (int k = 2; k <= n_pow2; k <<= 1) {
    int j = k >> 1;
    if (j >= 64) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kSortLdsRegs; ++r) {
        const int i = tid + 1024 * r;
        if (r < R && i < n_pow2) { keys[i] = kv[r]; ids[i] = iv[r]; }
      }
      __syncthreads();
      for (; j >= 64; j >>= 1) {
        for (int i = tid; i < n_pow2; i += blockDim.x) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const uint64_t ki = keys[i], kj = keys[ixj];
            const int32_t ii = ids[i], ij = ids[ixj];
            const bool gt = (ki > kj) || (ki == kj && ii > ij);
            const bool up = ((i & k) == 0);
            if (gt == up) {
              keys[i] = kj; keys[ixj] = ki;
              ids[i] = ij; ids[ixj] = ii;
            }
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < kSortLdsRegs; ++r) {
        const int i = tid + 1024 * r;
        if (r < R && i < n_pow2) { kv[r] = keys[i]; iv[r] = ids[i]; }
      }
    }
    for (; j > 0; j >>= 1) {
#pragma unroll
      for (int r = 0; r < kSortLdsRegs; ++r) {
        if (r < R) {
          const int i = tid + 1024 * r;
          const uint64_t pk = __shfl_xor(kv[r], j);
          const int32_t pi = __shfl_xor(iv[r], j);
          const bool gt = (kv[r] > pk) || (kv[r] == pk && iv[r] > pi);   // mine after partner's
          const bool lower = (i & j) == 0, up = (i & k) == 0;
          if (lower == up ? gt : !gt) { kv[r] = pk; iv[r] = pi; }
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortLdsRegs; ++r) {
    const int i = tid + 1024 * r;
    if (r < R && i < n_pow2) { keys[i] = kv[r]; ids[i] = iv[r]; }
  }
  __syncthreads();
}

// Log-spaced bins of a score's gap below the best score vmax: 64 bins per
// octave of g = vmax - v over [2^-32, 2^32) (the exponent and six leading
// mantissa bits of g), gaps below (and scores above vmax) to bin 0, above it
// and NaN to the last bin; non-decreasing as the score falls.  All scores in bins up to some b
// are at least as good as every score beyond it, so they form a prefix of the
// (score desc, id asc) order.
constexpr int kGapBins = 4096;
__device__ __forceinline__ int gap_bin(double vmax, double v) {
  const double g = vmax - v;           // >= 0 when vmax is the best (a bound above it: < 0)
  if (!(g == g)) return kGapBins - 1;
  if (!(g > 0.0)) return 0;
  const int e = (int)((unsigned)__double2hiint(g) >> 14) - ((1023 - 32) << 6);
  return e < 0 ? 0 : (e > kGapBins - 1 ? kGapBins - 1 : e);
}

// Inverse of desc_key (NaN came in as -inf).
__device__ __forceinline__ double key_value(uint64_t k) {
  const uint64_t sign = 0x8000000000000000ull;
  const uint64_t w = ~k;
  return __longlong_as_double((long long)((w & sign) ? (w ^ sign) : ~w));
}

// Second half of a radix-select step: hist holds the counts of the 8-bit
// digit at `shift` among the items with (key & pmask) == prefix; finds the
// digit holding the need-th smallest key and updates prefix and need.
// blockDim = 1024; ends with a barrier.
__device__ inline void radix_find(int shift, uint64_t &prefix, int &need, const unsigned *hist,
                                  uint64_t *sh_prefix, int *sh_need) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    // wave-parallel scan over the 256 digits: lane l owns digits 4l..4l+3
    unsigned h[4], own = 0u;
    for (int j = 0; j < 4; ++j) { h[j] = hist[4 * tid + j]; own += h[j]; }
    unsigned inc = own;
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned v = __shfl_up(inc, o);
      if (tid >= o) inc += v;
    }
    const unsigned excl = inc - own;
    const unsigned long long hit = __ballot(inc >= (unsigned)need);
    const int first = hit ? (__ffsll((long long)hit) - 1) : 63;
    if (tid == first) {
      unsigned cum = excl;
      int t = 4 * tid;
      for (int j = 0; j < 3; ++j, ++t) {
        if (cum + h[j] >= (unsigned)need) break;
        cum += h[j];
      }
      *sh_need = need - (int)cum;
      *sh_prefix = prefix | ((uint64_t)t << shift);
    }
  }
  __syncthreads();
  need = *sh_need;
  prefix = *sh_prefix;
  __syncthreads();
}

// One radix-select step: among the items with (key & pmask) == prefix, find
// the 8-bit digit at `shift` holding the need-th smallest key; updates prefix
// and need.  Keys come from key_at(i), i < n.  blockDim = 1024.
template <class KeyAt>
__device__ inline void radix_digit(int n, int shift, const KeyAt &key_at, uint64_t pmask,
                            uint64_t &prefix, int &need, unsigned *hist, uint64_t *sh_prefix,
                            int *sh_need) {
  const int tid = threadIdx.x;
  for (int i = tid; i < 256; i += blockDim.x) hist[i] = 0u;
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) {
    const uint64_t k = key_at(i);
    if ((k & pmask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  radix_find(shift, prefix, need, hist, sh_prefix, sh_need);
}

// Block-wide exclusive scan of non-negative counts (blockDim = 1024); returns
// the prefix and writes the block total to *total.
__device__ inline int block_excl_scan_count(int v, int *wsum, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  __syncthreads();
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  *total = tot;
  return off + inc - v;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o);
    v = (w < v) ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o);
    v = (w > v) ? w : v;
  }
  return v;
}

}  // namespace spg
