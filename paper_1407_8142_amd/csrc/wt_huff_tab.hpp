// Tables of a Huffman-shaped wavelet tree (byte alphabets), written by the
// build into a caller buffer and read by the queries.  See wt_huff.hpp for
// the shape and the level layout.
#pragma once

#include <stdint.h>

namespace wt {

constexpr int kHuffSyms = 256;
constexpr int kHuffMaxLevels = 48;  // n < 2^32 bounds the height by 45 (a depth-d leaf needs F(d+2) symbols)

struct HuffTab {
    uint32_t h, m, pad[2];            // height, symbols present
    uint64_t weight[kHuffSyms];       // occurrences per symbol
    uint32_t lens[kHuffSyms];         // code length per symbol (0: absent, or the only symbol)
    uint64_t codes[kHuffSyms];        // canonical code, left-aligned (bit 63 = code bit 0)
    uint32_t order[kHuffSyms];        // present symbols in (length, symbol) order
    uint64_t nd[kHuffMaxLevels];      // level sizes
    uint64_t ones[kHuffMaxLevels];    // ones per level
    // Level d, symbol c deeper than d: bit | next bit << 1 | continues << 2 | key << 8,
    // key = 2 * (index of c's node among the nodes of depth d, left to right) + bit.
    uint32_t lut[kHuffMaxLevels][kHuffSyms];
    uint32_t Dh[kHuffMaxLevels][2 * kHuffSyms];      // level-pass run destinations (wt_huff.hpp)
    uint64_t nstart[kHuffMaxLevels][kHuffSyms];      // start of node q in level d
    uint32_t child[kHuffMaxLevels][2 * kHuffSyms];   // child (q, b): its node index at d+1, or kHuffLeaf | symbol
};

constexpr uint32_t kHuffBit = 1u, kHuffNext = 2u, kHuffCont = 4u;
constexpr uint32_t kHuffLeaf = 0x80000000u;

}  // namespace wt
