// Iteration chunks of a CG solve between host convergence checks.
//
// The host reads the active-column flags after every chunk; iterations past
// convergence cost a launch each (their kernels exit at once), a check costs a
// stream synchronisation. A solve repeated every outer step takes about the
// same number of iterations each time, so the first chunk covers the previous
// count of the same solve and later chunks double from two iterations up to
// the check interval. Chunks are replayed from captured graphs of 2, 4, ...,
// 2^CHUNK_GRAPHS iterations (every chunk is even, so the two alternating
// scalar slots of the recurrence line up across graphs).
#pragma once

#include <algorithm>

namespace mlc {

constexpr int CHUNK_GRAPHS = 6;  // graphs of 2, 4, 8, 16, 32 and 64 iterations

// Length (even, >= 2) of chunk k of a solve; prev: length of chunk k - 1;
// predicted: iterations of the previous solve of this kind (0: none); every:
// the check interval (even).
inline int chunk_length(int k, int prev, int predicted, int every) {
  if (k == 0) return predicted > 0 ? std::max(2, (predicted + 1) & ~1) : every;
  return std::min(every, k == 1 ? 2 : 2 * prev);
}

// Calls f(g) for the graphs g (size 2 << g) that make up a chunk of L
// iterations, largest first.
template <class F>
void for_chunk_graphs(int L, F&& f) {
  constexpr int top = 2 << (CHUNK_GRAPHS - 1);
  for (; L >= top; L -= top) f(CHUNK_GRAPHS - 1);
  for (int g = CHUNK_GRAPHS - 1; g >= 0; --g)
    if (L & (2 << g)) f(g);
}

}  // namespace mlc
