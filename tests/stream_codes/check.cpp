// CPU check of the streamed-arc block coder (paper_1308_2144_amd/csrc/
// hb_stream_codes.h): random and extreme id sequences are coded block by
// block and read back with a decoder written here from the format's
// description (header byte, first id as a 7-bit variable-length integer,
// then zigzag differences as variable-length integers (header 0) or packed
// W = header - 1 bits wide, low bits first).  Prints "ok" when every block
// decodes to its ids, stays within its size bound, and takes the shorter of
// the two forms.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "hb_stream_codes.h"

namespace {

constexpr int kArcs = 32;

uint32_t get_varint(const std::vector<uint8_t>& b, size_t& at) {
  uint32_t v = 0;
  for (int shift = 0; shift < 35; shift += 7) {
    const uint32_t byte = b.at(at++);
    v |= (byte & 0x7fu) << shift;
    if (!(byte & 0x80u)) return v;
  }
  std::printf("varint longer than 5 bytes\n");
  std::exit(1);
}

uint32_t get_bits(const std::vector<uint8_t>& b, size_t base, uint64_t bit, int W) {
  uint64_t v = 0;
  for (int k = 0; k < W; ++k) {
    const uint64_t p = bit + (uint64_t)k;
    const uint32_t byte = b.at(base + (size_t)(p / 8));
    v |= (uint64_t)((byte >> (p % 8)) & 1u) << k;
  }
  return (uint32_t)v;
}

// Decodes one block of L ids starting at b[at]; returns the bytes it used.
size_t decode(const std::vector<uint8_t>& b, size_t at, int64_t L, std::vector<int32_t>& ids) {
  const size_t start = at;
  const uint32_t head = b.at(at++);
  uint32_t cur = get_varint(b, at);
  ids.push_back((int32_t)cur);
  if (head == 0) {
    for (int64_t a = 1; a < L; ++a) {
      const uint32_t z = get_varint(b, at);
      const int32_t d = (int32_t)((z >> 1) ^ (0u - (z & 1u)));
      cur += (uint32_t)d;
      ids.push_back((int32_t)cur);
    }
    return at - start;
  }
  const int W = (int)head - 1;
  if (W > 32) {
    std::printf("bad width %d\n", W);
    std::exit(1);
  }
  for (int64_t a = 1; a < L; ++a) {
    const uint32_t z = get_bits(b, at, (uint64_t)(a - 1) * (uint64_t)W, W);
    cur += (z >> 1) ^ (0u - (z & 1u));
    ids.push_back((int32_t)cur);
  }
  return at - start + (size_t)(((L - 1) * W + 7) / 8);
}

int check(const std::vector<int32_t>& ids, const char* what) {
  std::vector<uint8_t> bytes;
  std::vector<size_t> starts;
  for (size_t e = 0; e < ids.size(); e += kArcs) {
    starts.push_back(bytes.size());
    const int64_t L = (int64_t)std::min<size_t>(kArcs, ids.size() - e);
    const size_t before = bytes.size();
    hb::codes::put_block<kArcs>(bytes, ids.data() + e, L);
    const size_t used = bytes.size() - before;
    if (used > 1 + 5 * (size_t)L) {
      std::printf("%s: block of %lld ids took %zu bytes\n", what, (long long)L, used);
      return 1;
    }
  }
  std::vector<int32_t> back;
  for (size_t k = 0; k < starts.size(); ++k) {
    const int64_t L = (int64_t)std::min<size_t>(kArcs, ids.size() - k * kArcs);
    const size_t used = decode(bytes, starts[k], L, back);
    const size_t next = k + 1 < starts.size() ? starts[k + 1] : bytes.size();
    if (starts[k] + used != next) {
      std::printf("%s: block %zu used %zu bytes, stored %zu\n", what, k, used, next - starts[k]);
      return 1;
    }
    // the shorter form: sizes of both forms of this block, from the ids
    const int32_t* x = ids.data() + k * kArcs;
    auto vbytes = [](uint32_t v) { size_t n = 1; while (v >= 0x80u) { v >>= 7; ++n; } return n; };
    size_t var = 1 + vbytes((uint32_t)x[0]);
    int W = 0;
    for (int64_t a = 1; a < L; ++a) {
      const int32_t d = (int32_t)((uint32_t)x[a] - (uint32_t)x[a - 1]);
      const uint32_t z = ((uint32_t)d << 1) ^ (uint32_t)(d >> 31);
      var += vbytes(z);
      int w = 0;
      while (w < 32 && (z >> w) != 0u) ++w;
      W = std::max(W, w);
    }
    const size_t pk = 1 + vbytes((uint32_t)x[0]) + (size_t)(((L - 1) * W + 7) / 8);
    if (used != std::min(var, pk)) {
      std::printf("%s: block %zu took %zu bytes, forms %zu / %zu\n", what, k, used, var, pk);
      return 1;
    }
  }
  if (back != ids) {
    std::printf("%s: ids differ\n", what);
    return 1;
  }
  return 0;
}

}  // namespace

int main() {
  std::mt19937_64 rng(7);
  int bad = 0;
  // sorted rows of mixed lengths over a large id space (row starts jump)
  for (int t = 0; t < 200; ++t) {
    std::vector<int32_t> ids;
    const int rows = 1 + (int)(rng() % 40);
    for (int r = 0; r < rows; ++r) {
      const int len = 1 + (int)(rng() % (t % 2 ? 8 : 300));
      std::vector<int32_t> row;
      for (int k = 0; k < len; ++k) row.push_back((int32_t)(rng() % (1u << (10 + t % 22))));
      std::sort(row.begin(), row.end());
      ids.insert(ids.end(), row.begin(), row.end());
    }
    bad |= check(ids, "random rows");
  }
  // extremes: 0 and 2^31 - 1 alternating (widest differences), equal ids (zero
  // differences), single ids, one partial block
  std::vector<int32_t> ext;
  for (int k = 0; k < 97; ++k) ext.push_back(k % 2 ? 0x7fffffff : 0);
  bad |= check(ext, "alternating extremes");
  bad |= check(std::vector<int32_t>(70, 12345), "equal ids");
  bad |= check(std::vector<int32_t>{42}, "one id");
  std::vector<int32_t> up;
  for (int k = 0; k < 65; ++k) up.push_back(k * 3);
  bad |= check(up, "small gaps");
  std::vector<int32_t> down;
  for (int k = 0; k < 65; ++k) down.push_back(0x7fffffff - k * 1000003);
  bad |= check(down, "decreasing");
  if (bad) return 1;
  std::printf("ok\n");
  return 0;
}
