// Ladder initialisation: placement kernel (moves.hip) and the context
// accessors the host-side ladder initialisation (protocol.hip) uses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bpmf.h"
#include "internal.h"

namespace bpmf {

// Philox purpose of the initialisation draws; sub-purposes (purpose |
// sub << 8): SIR draws, site positions, orientations
enum : uint32_t { kInit = 7, kSubSir = 0, kSubCom = 1, kSubOrient = 2 };

// poses [first, first + count) of n_conf configurations confs (n_conf x n x
// 3) at n_com site positions x n_orient orientations, pose (c * n_com + i) *
// n_orient + o, written to out (count x n x 3); com: n_conf x 3 scratch
hipError_t launch_place_poses(const LigDev* lig, int n, const float* confs,
                              int n_conf, int n_com, int n_orient,
                              int64_t first, int64_t count, double* com,
                              uint64_t seed, float* out, hipStream_t st);

void* ctx_alloc(bpmf_ctx* c, size_t bytes);
void ctx_free(bpmf_ctx* c, void* p);
hipStream_t ctx_stream(bpmf_ctx* c);
uint64_t ctx_seed(bpmf_ctx* c);
int ctx_fail(int code, const char* msg);

}  // namespace bpmf
