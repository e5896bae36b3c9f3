// Host-side FFT planning: radix schedules, twiddle tables and launch shapes.
#pragma once

#include <stdint.h>

#include <vector>

#include "kernels.hpp"

namespace lshom {

// True if n factors over {2, 3, 5, 7}.
bool fft_size_ok(int64_t n);

// Default radix schedule for an axis of n points: radix 9 first, then
// 8, 7, 5, 6, 4, 3, 2 greedily.  An explicit schedule (autotuner) may replace it.
FftPlan default_plan(int n);

// Validates a caller-given schedule; fills plan on success.
bool make_plan(int n, const int* radices, int nstages, FftPlan* plan);

// exp(-2 pi i m / n), m in [0, n), evaluated in long double and rounded.
void twiddles(int n, std::vector<double>* re_im);

// Launch shape of the passes of one problem and precision.
struct PassShape {
  int rows_per_block;    // row pass (even)
  int tile0;             // axis-0 pass tile
  int tile1;             // axis-1 pass tile (3-D)
  int row_split;         // row pass: one component per block
  int threads_row;       // block size of the row pass (0: smallest that holds the batch)
  int threads_col;       // block size of the axis passes (0: as above)
};

// Default shapes within the FFT batch limit (256 threads) and lds_budget
// bytes of LDS, reduced while a pass would have fewer than min_blocks blocks.
// `transposed`: 2-D spectral arrays stored [k1][k0] (columns contiguous).
// `allow_split`: the row pass may hold one component per block (not for
// tensor phases, whose polarisation couples the components of a node).
PassShape default_shape(int d, const int64_t* N, const FftPlan* plans, int elem_bytes,
                        size_t lds_budget, long long min_blocks, bool transposed, int n_phases,
                        bool allow_split = true);

// True when every pass of the shape respects the FFT batch limit and the LDS
// budget (otherwise the problem is unsupported at this precision).
bool shape_fits(int d, const int64_t* N, const FftPlan* plans, const PassShape& s, int elem_bytes,
                size_t lds_budget, int n_phases);

}  // namespace lshom
