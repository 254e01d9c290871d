// Large-instance engine (placeholder until the multi-workgroup kernels land).
#pragma once

#include "lhdm_device.hpp"
#include "lhdm_host.hpp"

namespace lhdm {

static size_t large_workspace_bytes(int m, int n, int kmax) { return 0; }

static int large_solve(hipStream_t, int, int, const double*, long long, const double*, const DevParams&, double*,
                       double*, int*, lhdm_info*, void*, size_t) {
    return LHDM_EUNSUPPORTED;
}

}  // namespace lhdm
