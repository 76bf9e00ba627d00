// kernels.h -- host launchers of the PCBA kernels (internal).
#pragma once

#include <algorithm>

#include "pcba_internal.h"

namespace pcba {

// polynomials per root-conversion workgroup that fit LDS (0: none)
int root_run_length(int max_S, int tm_words);
hipError_t launch_reset_root(const DevInst* d_insts, int n, const int* d_pre, int total_blocks, int max_S,
                             int tm_words, int ppb, hipStream_t s);
hipError_t launch_racc(const DevInst* d_insts, int n, const int* d_pre, int total_polys, int max_S,
                       hipStream_t s);
hipError_t launch_plan(const DevInst* d_insts, int n, long long* plan, StepInfo* info, hipStream_t s);
// ev0/ev1 (or null): events stamped at the subdivision kernel's start and end.
// fuse (n <= PLAN_FUSE_MAX): the kernel forms the step's plan itself, in place
// of a k_plan launch before it, and writes it to plan / info.  tem / tpm: the
// largest tile (coefficients, patches) of the problems launched; nr: children
// regions per tile, 2, or NCMAX when some problem splits whole rounds; wg_cap:
// workgroups per compute unit at most (0: as many as fit).
// mfma: some FP32 problem of the launch splits on the matrix cores.
hipError_t launch_sub(const DevInst* d_insts, int n, long long* plan, StepInfo* info, bool fuse,
                      bool fp32, bool mfma, int maxm, int grid, int tem, int tpm, int nr, int wg_cap, hipStream_t s,
                      hipEvent_t ev0, hipEvent_t ev1);
// Up to n_steps whole steps (subdivision, cut) of a batch of one precision in
// one cooperative launch with grid barriers between the phases (n <=
// PLAN_FUSE_MAX, no FP32 re-derivation due within them).  bar: two device
// words (cleared here); herr: a host word the kernel sets to 1 if a barrier
// wait timed out.
hipError_t launch_steps(const DevInst* d_insts, int n, long long* plan, StepInfo* info, bool fp32, int maxm,
                        int tem, int tpm, int nr, int wg_cap, int n_steps, unsigned* bar, int* herr,
                        hipStream_t s);
// dynamic LDS bytes of k_sub for those tiles
size_t sub_lds_bytes(int tem, int tpm, bool fp32, int nr);
hipError_t launch_rederive(const DevInst* d_insts, int n, const long long* plan, const StepInfo* info,
                           int grid, int tgrid, size_t lds, hipStream_t s);
// max_children: an upper bound on the children (2K, or 2^l K in a round) at this
// step.  A problem with more than split (> 0) children is cut across workgroups
// of `part` children (four more launches, parts: at least
// n * ceil(max_children / part) records).
hipError_t launch_cut(const DevInst* d_insts, const StepInfo* info, int n, int64_t max_children,
                      long long split, int part, CutPart* parts, int64_t parts_cap, hipStream_t s);
hipError_t launch_gather(const DevInst* d_insts, int n, InstState* out, hipStream_t s);
// polynomials per certification workgroup that fit LDS (0: none)
int certify_run_length(int max_S, int tm_words);
hipError_t launch_certify(const DevInst* d_insts, int n, const int* d_pre, int total_blocks,
                          int max_S, int tm_words, int ppb, hipStream_t s);
hipError_t launch_pack(const DevInst& I, int K, double* out, uint32_t* ids, double* err, int64_t W,
                       hipStream_t s);

}  // namespace pcba
