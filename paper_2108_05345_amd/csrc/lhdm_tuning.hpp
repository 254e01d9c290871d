// Batched-engine table: written by paper_2108_05345_amd/autotune.py from
// timings on an MI355X (gfx950).  Rows are tried in order; the first whose
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
    {1e300, 1 << 30, 0},
};

}  // namespace lhdm
