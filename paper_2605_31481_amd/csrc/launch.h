// Kernel argument block and launcher declarations shared by the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "model.h"

namespace bard {

enum { OP_FK = 1, OP_JAC = 2, OP_RNEA = 4, OP_CRBA = 8 };

template <class Real>
struct Args {
  const Real* q;
  const Real* qd;
  const Real* qdd;
  const Real* tau_in;
  const Real* pi_ovr;
  Real* poses;
  Real* J;
  Real* tau;
  Real* M;
  Real* qdd_out;
  int64_t sq_b, sq_k, sqd_b, sqd_k, sqdd_b, sqdd_k, sti_b, sti_k;
  int64_t sp_b, sp_k, sJ_b, sJ_k, st_b, st_k, sM_b, sM_k, sqo_b, sqo_k;
  int64_t B;
  int logT;
  int log2P;  // lanes per instance of this launch, log2 (>= the model's minimum)
  int frame;
  int xcd_remap;
};

template <class Real, int OPS>
hipError_t launch_tree(const DevModel& dm, const DevEE& ee, const Args<Real>& ar, int grid, int block, size_t lds,
                       hipStream_t st);
template <class Real>
hipError_t launch_aba(const DevModel& dm, const Args<Real>& ar, int grid, int block, size_t lds, hipStream_t st);

}  // namespace bard
