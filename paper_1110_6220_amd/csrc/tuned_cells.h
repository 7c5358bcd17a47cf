// Cell sides chosen by paper_1110_6220_amd/autotune.py on AMD Radeon Graphics.
// Exact method only: its result does not depend on the cell side, so the
// table changes speed, never results.  Row: dtype (0 f64, 1 f32), batched
// (problems per launch > 1), largest side of the bucket, dense walls (wall
// density >= kDenseWalls), cell side.  Measurements (median of 3):
//   f64 batched=0 dense=0 n<=160 (4 problems, sides 33..160): 8: 2.27 ms, 16: 1.90 ms, 32: 1.96 ms, 64: 2.28 ms -> 16
//   f64 batched=1 dense=0 n<=160 (24 problems, sides 34..151): 8: 1.34 ms, 16: 0.95 ms, 32: 1.02 ms, 64: 1.24 ms -> 16
//   f64 batched=0 dense=0 n<=512 (4 problems, sides 161..512): 8: 5.80 ms, 16: 4.21 ms, 32: 3.82 ms, 64: 4.43 ms -> 32
//   f64 batched=1 dense=0 n<=512 (24 problems, sides 174..504): 8: 4.18 ms, 16: 2.72 ms, 32: 2.17 ms, 64: 2.15 ms -> 32
//   f64 batched=0 dense=0 n<=any (4 problems, sides 513..2049): 8: 29.94 ms, 16: 18.16 ms, 32: 14.08 ms, 64: 12.58 ms -> 64
//   f64 batched=1 dense=0 n<=any (12 problems, sides 650..1968): 8: 14.42 ms, 16: 8.40 ms, 32: 5.16 ms, 64: 5.21 ms -> 32
//   f64 batched=0 dense=1 n<=512 (3 problems, sides 159..430): 8: 7.41 ms, 16: 6.77 ms, 32: 8.72 ms, 64: 12.72 ms -> 16
//   f64 batched=1 dense=1 n<=512 (16 problems, sides 142..491): 8: 8.68 ms, 16: 6.24 ms, 32: 7.01 ms, 64: 10.81 ms -> 16
//   f64 batched=0 dense=1 n<=any (3 problems, sides 630..1048): 8: 61.48 ms, 16: 41.33 ms, 32: 40.38 ms, 64: 68.37 ms -> 32
//   f64 batched=1 dense=1 n<=any (16 problems, sides 630..1994): 8: 64.69 ms, 16: 45.50 ms, 32: 55.28 ms, 64: 81.07 ms -> 16
//   f32 batched=0 dense=0 n<=160 (4 problems, sides 33..160): 8: 2.25 ms, 16: 1.80 ms, 32: 1.89 ms, 64: 2.28 ms -> 16
//   f32 batched=1 dense=0 n<=160 (24 problems, sides 34..151): 8: 1.35 ms, 16: 0.96 ms, 32: 1.02 ms, 64: 1.29 ms -> 16
//   f32 batched=0 dense=0 n<=512 (4 problems, sides 161..512): 8: 5.75 ms, 16: 4.16 ms, 32: 3.72 ms, 64: 4.25 ms -> 32
//   f32 batched=1 dense=0 n<=512 (24 problems, sides 174..504): 8: 4.57 ms, 16: 2.75 ms, 32: 2.22 ms, 64: 2.34 ms -> 32
//   f32 batched=0 dense=0 n<=any (4 problems, sides 513..2049): 8: 29.40 ms, 16: 17.81 ms, 32: 13.71 ms, 64: 13.26 ms -> 64
//   f32 batched=1 dense=0 n<=any (12 problems, sides 650..1968): 8: 19.16 ms, 16: 8.84 ms, 32: 4.99 ms, 64: 5.27 ms -> 32
//   f32 batched=0 dense=1 n<=512 (3 problems, sides 159..430): 8: 7.17 ms, 16: 6.60 ms, 32: 8.28 ms, 64: 13.08 ms -> 16
//   f32 batched=1 dense=1 n<=512 (16 problems, sides 142..491): 8: 8.97 ms, 16: 6.41 ms, 32: 6.47 ms, 64: 11.39 ms -> 16
//   f32 batched=0 dense=1 n<=any (3 problems, sides 630..1048): 8: 52.52 ms, 16: 36.52 ms, 32: 37.08 ms, 64: 66.76 ms -> 16
//   f32 batched=1 dense=1 n<=any (16 problems, sides 630..1994): 8: 74.74 ms, 16: 49.26 ms, 32: 53.25 ms, 64: 77.87 ms -> 16
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
    {0, 1, 512, 0, 32},
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
