// Band widths of the band schedule, written by paper_1110_6220_amd/autotune.py
// (--bands).  Untuned defaults: one cell crossing at unit speed, the lowest
// band only.  Row: method (0 exact, 2 FHCM), dtype (0 f64, 1 f32), batched
// (problems per launch > 1), width in cell crossings s h, window.
#pragma once
namespace eik {
struct TunedBand {
  int method, dtype, batched;
  double factor;
  int window;
};
constexpr TunedBand kTunedBands[] = {
    {0, 0, 0, 1.0, 0}, {0, 0, 1, 1.0, 0}, {0, 1, 0, 1.0, 0}, {0, 1, 1, 1.0, 0},
    {2, 0, 0, 1.0, 0}, {2, 0, 1, 1.0, 0}, {2, 1, 0, 1.0, 0}, {2, 1, 1, 1.0, 0},
};
}  // namespace eik
