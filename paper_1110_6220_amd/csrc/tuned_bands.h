// Band widths of the band schedule, written by paper_1110_6220_amd/autotune.py
// (--bands) on AMD Radeon Graphics.  Row: method (0 exact, 2 FHCM), dtype
// (0 f64, 1 f32), batched (problems per launch > 1), width in cell
// crossings s h, window.  Measurements (median of 3; width/window: time,
// FHCM: max error / the heap order's, worse of 2 runs, must be <= 1.1):
//   exact f64 batched=0 (4 problems, sides 352..513): 0.5/0: 6.17 ms, 0.5/1: 4.89 ms, 0.5/3: 3.86 ms, 1/0: 5.26 ms, 1/1: 3.89 ms, 1/3: 3.55 ms, 2/0: 4.44 ms, 2/1: 3.51 ms, 2/3: 3.63 ms, 4/0: 4.03 ms, 4/1: 3.66 ms, 4/3: 3.52 ms, 8/0: 3.85 ms, 8/1: 3.55 ms, 8/3: 3.57 ms -> 2/1
//   exact f64 batched=1 (16 problems, sides 74..513): 0.5/0: 8.03 ms, 0.5/1: 4.59 ms, 0.5/3: 2.29 ms, 1/0: 6.45 ms, 1/1: 3.24 ms, 1/3: 1.98 ms, 2/0: 4.99 ms, 2/1: 2.51 ms, 2/3: 2.21 ms, 4/0: 4.31 ms, 4/1: 2.55 ms, 4/3: 2.31 ms, 8/0: 3.98 ms, 8/1: 2.81 ms, 8/3: 2.67 ms -> 1/3
//   exact f32 batched=0 (4 problems, sides 352..513): 0.5/0: 5.73 ms, 0.5/1: 4.34 ms, 0.5/3: 3.19 ms, 1/0: 4.71 ms, 1/1: 3.36 ms, 1/3: 2.91 ms, 2/0: 3.91 ms, 2/1: 2.90 ms, 2/3: 2.85 ms, 4/0: 3.61 ms, 4/1: 2.87 ms, 4/3: 2.89 ms, 8/0: 3.11 ms, 8/1: 2.92 ms, 8/3: 2.92 ms -> 2/3
//   exact f32 batched=1 (16 problems, sides 74..513): 0.5/0: 7.60 ms, 0.5/1: 4.41 ms, 0.5/3: 2.22 ms, 1/0: 5.92 ms, 1/1: 3.02 ms, 1/3: 1.84 ms, 2/0: 4.49 ms, 2/1: 2.28 ms, 2/3: 1.97 ms, 4/0: 4.05 ms, 4/1: 2.30 ms, 4/3: 2.08 ms, 8/0: 3.56 ms, 8/1: 2.78 ms, 8/3: 2.57 ms -> 1/3
//   fhcm f64 batched=0 (4 problems, sides 352..513): 0.5/0: 6.60 ms err x1.00, 0.5/1: 4.48 ms err x1.00, 0.5/3: 3.21 ms err x1.00, 1/0: 5.09 ms err x1.00, 1/1: 3.15 ms err x1.00, 1/3: 2.51 ms err x1.00, 2/0: 4.27 ms err x1.00, 2/1: 2.61 ms err x1.00, 2/3: 2.43 ms err x1.34, 4/0: 3.27 ms err x0.80, 4/1: 2.44 ms err x0.74, 4/3: 2.48 ms err x0.54, 8/0: 2.65 ms err x0.74, 8/1: 2.51 ms err x0.54, 8/3: 2.62 ms err x0.54 -> 4/1
//   fhcm f64 batched=1 (16 problems, sides 91..499): 0.5/0: 4.36 ms err x0.60, 0.5/1: 2.60 ms err x0.60, 0.5/3: 1.66 ms err x0.60, 1/0: 3.37 ms err x0.17, 1/1: 1.89 ms err x0.17, 1/3: 1.38 ms err x0.60, 2/0: 2.72 ms err x0.60, 2/1: 1.64 ms err x0.60, 2/3: 1.28 ms err x0.60, 4/0: 2.21 ms err x0.60, 4/1: 1.44 ms err x0.60, 4/3: 1.36 ms err x0.60, 8/0: 1.90 ms err x0.60, 8/1: 1.43 ms err x0.60, 8/3: 1.46 ms err x0.60 -> 2/3
//   fhcm f32 batched=0 (4 problems, sides 352..513): 0.5/0: 5.92 ms err x1.00, 0.5/1: 3.96 ms err x1.00, 0.5/3: 2.55 ms err x1.00, 1/0: 4.45 ms err x1.00, 1/1: 2.76 ms err x1.00, 1/3: 2.29 ms err x1.00, 2/0: 3.78 ms err x1.00, 2/1: 2.34 ms err x1.00, 2/3: 2.13 ms err x1.00, 4/0: 2.82 ms err x0.80, 4/1: 2.26 ms err x0.74, 4/3: 2.24 ms err x0.74, 8/0: 2.42 ms err x0.74, 8/1: 2.30 ms err x0.39, 8/3: 2.27 ms err x0.54 -> 2/3
//   fhcm f32 batched=1 (16 problems, sides 91..499): 0.5/0: 6.69 ms err x0.60, 0.5/1: 3.82 ms err x0.60, 0.5/3: 2.15 ms err x0.21, 1/0: 5.37 ms err x0.28, 1/1: 2.51 ms err x0.17, 1/3: 1.94 ms err x0.60, 2/0: 4.22 ms err x0.28, 2/1: 2.23 ms err x0.60, 2/3: 1.75 ms err x0.60, 4/0: 3.70 ms err x0.60, 4/1: 2.33 ms err x0.28, 4/3: 2.22 ms err x0.60, 8/0: 3.19 ms err x0.60, 8/1: 2.35 ms err x0.60, 8/3: 2.15 ms err x0.60 -> 2/3
#pragma once
namespace eik {
struct TunedBand {
  int method, dtype, batched;
  double factor;
  int window;
};
constexpr TunedBand kTunedBands[] = {
    {0, 0, 0, 2.0, 1},
    {0, 0, 1, 1.0, 3},
    {0, 1, 0, 2.0, 3},
    {0, 1, 1, 1.0, 3},
    {2, 0, 0, 4.0, 1},
    {2, 0, 1, 2.0, 3},
    {2, 1, 0, 2.0, 3},
    {2, 1, 1, 2.0, 3},
};
}  // namespace eik
