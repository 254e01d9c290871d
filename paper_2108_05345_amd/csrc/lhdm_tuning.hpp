// Batched-engine table: written by paper_2108_05345_amd/autotune.py from
// timings on AMD Radeon Graphics (gfx950, 256 CUs).  Rows are tried in order; the first whose
// bounds hold gives the engine (0: fused, one workgroup per compute unit;
// 1: fused, two per compute unit; 2: phased).
#pragma once

namespace lhdm {

struct TuneRow {
    double per_cu_hi;   // instances per compute unit <= this
    int m_hi;           // largest m of the batch <= this
    int engine;
};

static const TuneRow kTuneRows[] = {
    {0.25, 64, 1},
    {0.25, 128, 0},
    {0.25, 256, 0},
    {0.25, 512, 0},
    {0.25, 1024, 0},
    {0.5, 64, 0},
    {0.5, 128, 0},
    {0.5, 256, 0},
    {0.5, 512, 0},
    {0.5, 1024, 0},
    {1.0, 64, 0},
    {1.0, 128, 0},
    {1.0, 256, 0},
    {1.0, 512, 0},
    {2.0, 64, 1},
    {2.0, 128, 1},
    {2.0, 256, 1},
    {2.0, 512, 1},
    {4.0, 64, 1},
    {4.0, 128, 1},
    {4.0, 256, 1},
    {8.0, 64, 1},
    {8.0, 128, 1},
    {8.0, 256, 1},
    {1e300, 1 << 30, 0},
};

}  // namespace lhdm
