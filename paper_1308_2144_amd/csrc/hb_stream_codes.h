// Host-side coding of the arc blocks of compressed streamed graphs
// (opt.stream_compress); k_decode_chunk reads the same format.  A block holds
// L <= MaxArcs consecutive successor ids: a header byte, the first id as a
// variable-length integer (7 bits per byte, low bits first, high bit set on
// every byte but the last), then the zigzag-coded differences of consecutive
// ids, either as variable-length integers too (header 0) or bit-packed at the
// block's widest difference W, low bits first (header W + 1), whichever is
// shorter: gaps inside a sorted row are alike in size, so packing saves the
// 7-bit granularity, while blocks of short rows, with a random jump at every
// row start, keep the variable lengths.  Host-only, no HIP.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace hb {
namespace codes {

inline void put_varint(std::vector<uint8_t>& out, uint32_t v) {
  while (v >= 0x80u) {
    out.push_back((uint8_t)(v | 0x80u));
    v >>= 7;
  }
  out.push_back((uint8_t)v);
}

inline int varint_len(uint32_t v) {
  int k = 1;
  while (v >= 0x80u) {
    v >>= 7;
    ++k;
  }
  return k;
}

inline int bit_width(uint32_t v) { return v == 0u ? 0 : 32 - __builtin_clz(v); }

// Appends the block of ids x[0..L) to out (1 <= L <= MaxArcs).
template <int MaxArcs>
inline void put_block(std::vector<uint8_t>& out, const int32_t* x, int64_t L) {
  uint32_t z[MaxArcs];
  int64_t vlen = 0;
  int W = 0;
  for (int64_t a = 1; a < L; ++a) {
    const int32_t d = (int32_t)((uint32_t)x[a] - (uint32_t)x[a - 1]);
    z[a] = ((uint32_t)d << 1) ^ (uint32_t)(d >> 31);
    vlen += varint_len(z[a]);
    W = std::max(W, bit_width(z[a]));
  }
  const int64_t plen = ((L - 1) * W + 7) / 8;
  const bool packed = plen < vlen;
  out.push_back(packed ? (uint8_t)(W + 1) : (uint8_t)0);
  put_varint(out, (uint32_t)x[0]);
  if (!packed) {
    for (int64_t a = 1; a < L; ++a) put_varint(out, z[a]);
    return;
  }
  uint64_t acc = 0;
  int nbits = 0;
  for (int64_t a = 1; a < L; ++a) {
    acc |= (uint64_t)z[a] << nbits;
    nbits += W;
    while (nbits >= 8) {
      out.push_back((uint8_t)acc);
      acc >>= 8;
      nbits -= 8;
    }
  }
  if (nbits > 0) out.push_back((uint8_t)acc);
}

}  // namespace codes
}  // namespace hb
