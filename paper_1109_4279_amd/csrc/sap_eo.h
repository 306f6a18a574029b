// Pieces of the even/odd block solver: the DPP exchange between the two lanes of a site
// pair and the clover blocks of the even/odd clover field (A on even sites, A^-1 on odd
// sites).
#pragma once

#include "wc_kernels.h"

namespace wc {

// value of the partner lane (lane ^ 1) by a DPP quad permutation [1, 0, 3, 2]: a VALU move,
// no LDS round trip.  Every lane of the wavefront must execute it.
WC_D float xor1(float v) { return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false)); }
WC_D double xor1(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <class R> WC_D cplx<R> shfl1(cplx<R> v) { return {xor1(v.re), xor1(v.im)}; }

// clover block blk (runtime) of the even/odd clover field, scale not applied
template <int P, class R>
WC_D Herm6<R> clover_block(const LatDesc& L, int V, int site, int blk) {
  if constexpr (P == P_F64 || P == P_F32) {
    return CloverIO<P>::load_raw(L.clov_eo, L.cscale_eo, V, site, blk);
  } else {
    // 72 halves per site in 9 uint4; block 0 is halves 0..35 of uint4 0..4, block 1 is
    // halves 4..39 of uint4 4..8: load five uint4 from 4*blk and take the block's 18 words
    // (a word-level select: block 1 starts two words in)
    const size_t p = (size_t)site + (size_t)(4 * blk) * V;
    uint32_t wd[20];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const uint4 v = gld_u4(L.clov_eo, p + (size_t)k * V);
      wd[4 * k] = v.x;
      wd[4 * k + 1] = v.y;
      wd[4 * k + 2] = v.z;
      wd[4 * k + 3] = v.w;
    }
    float H[36];
#pragma unroll
    for (int j = 0; j < 18; ++j) {
      const uint32_t u = blk ? wd[j + 2] : wd[j];
      H[2 * j] = s16_to_f32<P>(uint16_t(u & 0xFFFFu));
      H[2 * j + 1] = s16_to_f32<P>(uint16_t(u >> 16));
    }
    Herm6<R> h;
#pragma unroll
    for (int i = 0; i < 6; ++i) h.d[i] = H[i];
#pragma unroll
    for (int k = 0; k < 15; ++k) h.o[k] = {H[6 + 2 * k], H[7 + 2 * k]};
    return h;
  }
}

// the storage scale of clover block blk (1 for FP64 / FP32 storage)
template <int P, class R>
WC_D R clover_scale(const LatDesc& L, int site, int blk) {
  return CloverIO<P>::scale(L.cscale_eo, site, blk);
}

template <int P, class R>
WC_D Herm6<R> clover_block_scaled(const LatDesc& L, int V, int site, int blk) {
  Herm6<R> h = clover_block<P, R>(L, V, site, blk);
  const R cs = clover_scale<P, R>(L, site, blk);
  if (P == P_F16 || P == P_BF16) {
#pragma unroll
    for (int i = 0; i < 6; ++i) h.d[i] *= cs;
#pragma unroll
    for (int k = 0; k < 15; ++k) h.o[k] = cs * h.o[k];
  }
  return h;
}

}  // namespace wc
