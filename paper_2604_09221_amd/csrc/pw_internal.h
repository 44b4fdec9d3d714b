// pw_internal.h -- layout of the per-triangulation "program" that the scheme
// kernels walk, shared by the host builder (tri.cpp) and the kernels.
//
// The reflected diamond A<> (Sec. 2) is numbered row by row (y ascending,
// then x ascending).  Every diamond edge is listed once, at its later
// endpoint, so the kernels can process vertices in order and only ever look
// back.  All of it is read with wave-uniform loads (scalar cache).
//
//   words [0, nV)                   vertex records
//       bits  0..6   p   : lattice point (|x|,|y|) index k in A (mask bit)
//       bit   7      g   : reflection parity [x<0]|x| + [y<0]|y| mod 2,
//                          so sign(v) = bit p of the mask XOR g (eq. (signs))
//       bits  8..15  n   : number of earlier neighbours
//       bits 16..31  off : offset of the first earlier neighbour in the list
//   words [nV, nV+nE)               earlier-neighbour ids (one per word)
//   words [nV+nE, nV+nE+nP)         antipodal pairs a | b << 16, a < b
#pragma once
#if !defined(__HIPCC_RTC__)
#include <cstdint>
#endif

namespace pw {

constexpr int kDMax = 12;
constexpr int kVMax = 2 * kDMax * kDMax + 2 * kDMax + 1;  // 313
constexpr int kEMax = 6 * kDMax * kDMax + 2 * kDMax;      // 888

constexpr int n_points(int d) { return (d + 1) * (d + 2) / 2; }
constexpr int n_vertices(int d) { return 2 * d * d + 2 * d + 1; }
constexpr int n_diamond_edges(int d) { return 6 * d * d + 2 * d; }
constexpr int harnack(int d) { return (d - 1) * (d - 2) / 2 + 1; }
constexpr int mask_bytes(int d) { return n_points(d) <= 32 ? 4 : (n_points(d) <= 64 ? 8 : 16); }

// device-side error flags (sticky, per triangulation handle)
constexpr uint32_t kErrRegions = 1u;   // more regions than Harnack's bound
constexpr uint32_t kErrRoot = 2u;      // no unique root
constexpr uint32_t kErrTree = 4u;      // adjacency graph is not a tree
constexpr uint32_t kErrSelfLoop = 8u;  // self-loop for even d
constexpr uint32_t kErrOverflow = 16u;  // more regions than capped tables hold (not an error of the input)

// Lane groups (the batched launch): G = 2 or 4 lanes evaluate one mask, each
// on one block of the diamond -- the upper half y >= 0 (G = 2) or the
// quadrant x, y >= 0 (G = 4) -- reflected for lane q = sx + 2 sy (G = 4) or
// q = sy (G = 2) into the block (-1)^sx x, (-1)^sy y.  Block vertices are
// numbered in diamond order (y, then x); vertex v of lane q has the group
// index v * G + q.  A group program is
//   words [0, NB)         vertex records: p | g << 7 | n << 8 | off << 16,
//                         with off in bits 16..27, bit 28 = (x == 0),
//                         bit 29 = (y == 0) (block coordinates)
//   words [NB, NB+NEB)    earlier neighbours: block id | (p | g << 7) << 16
//   words [.., +NGL)      glues a | b << 16 (group indices, a < b): the
//                         copies of an axis point in two blocks
//   words [.., +2d)       antipodal pairs a | b << 16 (group indices)
// A copy of an axis point in block q is glued to the copy in block
// q - 1 if sx = 1 and x = 0 (G = 4), else to the copy in block q - 2
// (G = 4) or q - 1 (G = 2) if sy = 1 and y = 0.
constexpr int group_block_vertices(int d, int g) { return g == 4 ? n_points(d) : (d + 1) * (d + 1); }
constexpr int group_block_edges(int d, int g) {
  return g == 4 ? n_points(d) + d * d - 1 : 2 * (n_points(d) + d * d - 1) - d;
}
constexpr int group_glues(int d, int g) { return g == 4 ? 4 * d + 3 : 2 * d + 1; }
constexpr int group_program_words(int d, int g) {
  return group_block_vertices(d, g) + group_block_edges(d, g) + group_glues(d, g) + 2 * d;
}
constexpr int kGroupMinDegree = 8;  // lane groups serve degrees 8..12 (u16 entries)
constexpr int kGroupWordsMax = group_program_words(kDMax, 2) > group_program_words(kDMax, 4)
                                   ? group_program_words(kDMax, 2)
                                   : group_program_words(kDMax, 4);

#if !defined(__HIPCC_RTC__)
struct HostProgram {
  int d = 0, nA = 0, nV = 0, nE = 0, nP = 0;
  std::uint32_t words[kVMax + kEMax + 2 * kDMax];
  int n_words = 0;
};

// Validates the edge list and fills `prog`.  Returns 0 or a negative
// pw_status, with a message in `err`.
int build_program(int d, const int16_t* edges_ij, int n_edges, HostProgram* prog, char* err, int errlen);

// The group program for G = 2 or 4 lanes per mask, derived from a diamond
// program (d >= 2).  words must hold group_program_words(d, G).  Returns 0
// or a negative pw_status, with a message in `err`.
int build_group_program(const HostProgram& full, int G, std::uint32_t* words, char* err, int errlen);
#endif

}  // namespace pw
