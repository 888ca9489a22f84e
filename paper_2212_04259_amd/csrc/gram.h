// Shared pieces of the one-hot Gram contractions on gfx950 int8 MFMA (depth
// 0 over all variables, depth 1 over each node's neighbours under a mask):
// operand types, the workgroup size and the one-hot expansion of uint8
// columns.
#pragma once

#include "device_ci.h"

namespace bns {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kGramWG = 256;

// One-hot bytes [b == cat] of the 16 samples in w; bytes at and beyond
// nvalid are zero.  Variables of at most 8 categories take one byte permute
// per 4 samples (the sample bytes select from a pool whose byte cat is 1);
// wider ones an exact zero-byte test of w ^ cat.
BNS_INLINE u32x4 onehot16(u32x4 w, uint32_t plo, uint32_t phi, uint32_t cat, bool wide, int nvalid) {
    u32x4 o;
    // (one branch for the four words: the wide form is rare)
    if (!wide) {
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = __builtin_amdgcn_perm(phi, plo, w[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t d = w[k] ^ (cat * 0x01010101u);
            const uint32_t t = ~(((d & 0x7f7f7f7fu) + 0x7f7f7f7fu) | d | 0x7f7f7f7fu);
            o[k] = t >> 7;
        }
    }
    // (only the last group of a chunk is partial: whole groups skip the masks)
    if (nvalid < 16) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int vk = nvalid - 4 * k;
            const uint32_t keep = vk >= 4 ? 0xffffffffu : vk <= 0 ? 0u : ((1u << (8 * vk)) - 1u);
            o[k] &= keep;
        }
    }
    return o;
}

}  // namespace bns
