// Cell sides chosen by paper_1110_6220_amd/autotune.py on AMD Radeon Graphics.
// Exact method only: its result does not depend on the cell side, so the
// table changes speed, never results.  Row: dtype (0 f64, 1 f32), batched
// (problems per launch > 1), largest side of the bucket, dense walls (wall
// density >= kDenseWalls), cell side.  Measurements (median of 3):
//   f64 batched=0 dense=0 n<=160 (4 problems, sides 33..160): 8: 2.30 ms, 16: 1.96 ms, 32: 2.04 ms, 64: 2.34 ms -> 16
//   f64 batched=1 dense=0 n<=160 (24 problems, sides 34..151): 8: 1.35 ms, 16: 0.99 ms, 32: 1.06 ms, 64: 1.27 ms -> 16
//   f64 batched=0 dense=0 n<=512 (4 problems, sides 161..512): 8: 5.86 ms, 16: 4.29 ms, 32: 3.88 ms, 64: 4.50 ms -> 32
//   f64 batched=1 dense=0 n<=512 (24 problems, sides 174..504): 8: 4.26 ms, 16: 2.74 ms, 32: 2.17 ms, 64: 2.16 ms -> 64
//   f64 batched=0 dense=0 n<=any (4 problems, sides 513..2049): 8: 29.97 ms, 16: 18.20 ms, 32: 14.09 ms, 64: 12.61 ms -> 64
//   f64 batched=1 dense=0 n<=any (12 problems, sides 650..1968): 8: 14.70 ms, 16: 8.54 ms, 32: 5.19 ms, 64: 5.19 ms -> 32
//   f64 batched=0 dense=1 n<=512 (3 problems, sides 159..430): 8: 7.36 ms, 16: 6.73 ms, 32: 8.77 ms, 64: 12.68 ms -> 16
//   f64 batched=1 dense=1 n<=512 (16 problems, sides 142..491): 8: 8.78 ms, 16: 6.45 ms, 32: 7.02 ms, 64: 11.13 ms -> 16
//   f64 batched=0 dense=1 n<=any (3 problems, sides 630..1048): 8: 65.11 ms, 16: 41.17 ms, 32: 39.90 ms, 64: 68.07 ms -> 32
//   f64 batched=1 dense=1 n<=any (16 problems, sides 630..1994): 8: 66.44 ms, 16: 46.59 ms, 32: 56.15 ms, 64: 82.57 ms -> 16
//   f32 batched=0 dense=0 n<=160 (4 problems, sides 33..160): 8: 2.24 ms, 16: 1.79 ms, 32: 1.88 ms, 64: 2.29 ms -> 16
//   f32 batched=1 dense=0 n<=160 (24 problems, sides 34..151): 8: 1.36 ms, 16: 0.96 ms, 32: 1.04 ms, 64: 1.31 ms -> 16
//   f32 batched=0 dense=0 n<=512 (4 problems, sides 161..512): 8: 5.76 ms, 16: 4.19 ms, 32: 3.73 ms, 64: 4.26 ms -> 32
//   f32 batched=1 dense=0 n<=512 (24 problems, sides 174..504): 8: 4.60 ms, 16: 2.72 ms, 32: 2.18 ms, 64: 2.29 ms -> 32
//   f32 batched=0 dense=0 n<=any (4 problems, sides 513..2049): 8: 29.38 ms, 16: 17.79 ms, 32: 13.69 ms, 64: 13.26 ms -> 64
//   f32 batched=1 dense=0 n<=any (12 problems, sides 650..1968): 8: 19.64 ms, 16: 8.97 ms, 32: 5.00 ms, 64: 5.27 ms -> 32
//   f32 batched=0 dense=1 n<=512 (3 problems, sides 159..430): 8: 7.22 ms, 16: 6.64 ms, 32: 8.41 ms, 64: 13.04 ms -> 16
//   f32 batched=1 dense=1 n<=512 (16 problems, sides 142..491): 8: 9.16 ms, 16: 6.47 ms, 32: 6.50 ms, 64: 11.34 ms -> 16
//   f32 batched=0 dense=1 n<=any (3 problems, sides 630..1048): 8: 50.77 ms, 16: 36.39 ms, 32: 36.84 ms, 64: 68.02 ms -> 16
//   f32 batched=1 dense=1 n<=any (16 problems, sides 630..1994): 8: 73.65 ms, 16: 50.24 ms, 32: 53.47 ms, 64: 77.91 ms -> 16
#pragma once
namespace eik {
constexpr double kDenseWalls = 0.03;
struct TunedCell {
  int dtype, batched, nmax, dense, cell;
};
constexpr TunedCell kTunedCells[] = {
    {0, 0, 160, 0, 16},
    {0, 1, 160, 0, 16},
    {0, 0, 512, 0, 32},
    {0, 1, 512, 0, 64},
    {0, 0, 1 << 30, 0, 64},
    {0, 1, 1 << 30, 0, 32},
    {0, 0, 512, 1, 16},
    {0, 1, 512, 1, 16},
    {0, 0, 1 << 30, 1, 32},
    {0, 1, 1 << 30, 1, 16},
    {1, 0, 160, 0, 16},
    {1, 1, 160, 0, 16},
    {1, 0, 512, 0, 32},
    {1, 1, 512, 0, 32},
    {1, 0, 1 << 30, 0, 64},
    {1, 1, 1 << 30, 0, 32},
    {1, 0, 512, 1, 16},
    {1, 1, 512, 1, 16},
    {1, 0, 1 << 30, 1, 16},
    {1, 1, 1 << 30, 1, 16},
};
}  // namespace eik
