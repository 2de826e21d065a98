// Wavefront sums of FP64 values without LDS (row-swap permutes and DPP), shared by
// the vector kernels and the residual kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace frjf {

// Workgroup i of T runs on XCD i % 8; the work item it takes is xcd_remap(i, T), so
// each XCD takes one contiguous range of items (neighbouring tiles, or the same range
// of vector entries in every kernel of a chain) and they share its L2.  A bijection
// on [0, T).
__device__ __forceinline__ int xcd_remap(int i, int T) {
  const int q = T >> 3, r = T & 7;
  const int x = i & 7, l = i >> 3;
  return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// ---------------------------------------------------------------- wavefront sums
// Lane exchanges without LDS, in six stages that each pair a lane with one whose
// set of already summed lanes is disjoint from its own: stage 0 pairs lanes 32
// apart and stage 1 lanes 16 apart (row-swap permutes), stages 2..5 work inside a
// 16-lane row by DPP (rotate by 8, mirror inside 8 lanes, quad permutes 2 and 1
// apart).  Stage S splits the pairs by lane bit 5 - S into a lower and an upper
// lane.

__device__ __forceinline__ unsigned lo32(double x) { return (unsigned)__double2loint(x); }
__device__ __forceinline__ unsigned hi32(double x) { return (unsigned)__double2hiint(x); }
__device__ __forceinline__ double mk64(unsigned hi, unsigned lo) { return __hiloint2double((int)hi, (int)lo); }

// Swap stage S < 2: the lower lane of a pair gets a(own) + a(partner), the upper
// one b(partner) + b(own).
template <int S>
__device__ __forceinline__ double swap_add(double a, double b) {
  if constexpr (S == 0) {
    const auto rl = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
    return mk64(rh[0], rl[0]) + mk64(rh[1], rl[1]);
  } else {
    const auto rl = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
    return mk64(rh[0], rl[0]) + mk64(rh[1], rl[1]);
  }
}

// DPP stage 2 <= S < 6: the partner's x
template <int S>
__device__ __forceinline__ double dpp_partner(double x) {
  constexpr int CTRL = S == 2 ? 0x128 : (S == 3 ? 0x141 : (S == 4 ? 0x4e : 0xb1));
  const int l = __builtin_amdgcn_update_dpp((int)lo32(x), (int)lo32(x), CTRL, 0xf, 0xf, false);
  const int h = __builtin_amdgcn_update_dpp((int)hi32(x), (int)hi32(x), CTRL, 0xf, 0xf, false);
  return mk64((unsigned)h, (unsigned)l);
}

// Values each lane holds after wave_multi_sum of K values: a stage halves an even
// count (each lane of a pair keeps half of the sums) and sums an odd one in full.
constexpr int multi_sum_count(int K, int s = 0) {
  return s == 6 ? K : multi_sum_count(K % 2 == 0 ? K / 2 : K, s + 1);
}

template <int S, int KC, int K>
__device__ __forceinline__ void multi_sum(double (&a)[K], int lane, int& off, int& full) {
  if constexpr (S < 6) {
    constexpr int BIT = 5 - S;
    const bool up = (lane >> BIT) & 1;
    if constexpr (KC % 2 == 0) {
      constexpr int H = KC / 2;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        if constexpr (S < 2) {
          a[i] = swap_add<S>(a[i], a[i + H]);
        } else {
          const double send = up ? a[i] : a[i + H];
          const double keep = up ? a[i + H] : a[i];
          a[i] = keep + dpp_partner<S>(send);
        }
      }
      if (up) off += H;
      multi_sum<S + 1, H>(a, lane, off, full);
    } else {
#pragma unroll
      for (int i = 0; i < KC; ++i) {
        if constexpr (S < 2)
          a[i] = swap_add<S>(a[i], a[i]);
        else
          a[i] += dpp_partner<S>(a[i]);
      }
      full |= 1 << BIT;
      multi_sum<S + 1, KC>(a, lane, off, full);
    }
  }
}

// Sums of a[t], t < K, over the wavefront, about K + 6 exchanges instead of 6 K.
// Afterwards a[0 .. multi_sum_count(K) - 1] of a lane hold the sums of
// t = off .. off + multi_sum_count(K) - 1; exactly one lane per range returns true.
template <int K>
__device__ __forceinline__ bool wave_multi_sum(double (&a)[K], int& off) {
  const int lane = threadIdx.x & 63;
  int full = 0;
  off = 0;
  multi_sum<0, K>(a, lane, off, full);
  return (lane & full) == 0;
}

// Sum of v over the wavefront, in every lane
__device__ __forceinline__ double wave_sum(double v) {
  double a[1] = {v};
  int off;
  wave_multi_sum<1>(a, off);
  return a[0];
}

// Sum of the nb partial sums p[0 .. nb), computed by every wavefront on its own in one
// fixed order (so every wavefront of every workgroup gets the same bits): lane l adds
// p[l], p[l + 64], ..., then the lanes are summed.
__device__ __forceinline__ double wave_sum_partials(const double* __restrict__ p, int nb) {
  const int lane = threadIdx.x & 63;
  double a[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) a[q] = (lane + 64 * q < nb) ? p[lane + 64 * q] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) s += a[q];
  for (int b = lane + 64 * 16; b < nb; b += 64) s += p[b];
  return wave_sum(s);
}

}  // namespace frjf
