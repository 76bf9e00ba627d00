// kernels.h -- host launchers of the PCBA kernels (internal).
#pragma once

#include <algorithm>

#include "pcba_internal.h"

namespace pcba {

hipError_t launch_root(const DevInst& I, const double* mono, const double* mats, const int* matoff,
                       double* root, double* root_err, int64_t W, int max_S, hipStream_t s);
hipError_t launch_plan(const DevInst* d_insts, int n, long long* plan, hipStream_t s);
hipError_t launch_sub(const DevInst* d_insts, int n, const long long* plan, bool fp32, int maxm,
                      int grid, size_t lds, hipStream_t s);
hipError_t launch_rederive(const DevInst* d_insts, int n, const long long* plan, int grid,
                           size_t lds, hipStream_t s);
hipError_t launch_cut(const DevInst* d_insts, int n, hipStream_t s);
hipError_t launch_gather(const DevInst* d_insts, int n, InstState* out, hipStream_t s);
hipError_t launch_certify(const DevInst& I, int max_S, int max_m, hipStream_t s);
hipError_t launch_pack(const DevInst& I, int K, double* out, uint32_t* ids, double* err, int64_t W,
                       hipStream_t s);

}  // namespace pcba
