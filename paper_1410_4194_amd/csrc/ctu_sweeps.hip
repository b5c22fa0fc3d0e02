// ctu_sweeps.hip -- instantiates the sweep kernels for one storage type and solver class.
// The build compiles this file once per (CTU_SWEEP_T, CTU_SWEEP_K) pair, in parallel: double
// and float, each with the exact solver for K = 0 (any gamma), 3 (gamma = 5/3) and
// 5 (gamma = 7/5), and with the Roe solver (K = kRoe = 1).
#include "ctu_sweeps.hpp"

#if !defined(CTU_SWEEP_T) || !defined(CTU_SWEEP_K)
#error "compile with -DCTU_SWEEP_T=<double|float> -DCTU_SWEEP_K=<0|1|3|5>"
#endif

namespace ctu {

template <>
hipError_t launch_sweeps<CTU_SWEEP_T, CTU_SWEEP_K>(const PlanView& v, int stage, hipStream_t stream,
                                                   Profiler* prof) {
  // the Newton histogram exists for the exact solver only
  if constexpr (CTU_SWEEP_K != kRoe) {
    if (prof && prof->hist) {
      enqueue_sweeps<CTU_SWEEP_T, CTU_SWEEP_K, true>(v, stage, stream, prof);
      return hipGetLastError();
    }
  }
  enqueue_sweeps<CTU_SWEEP_T, CTU_SWEEP_K, false>(v, stage, stream, prof);
  return hipGetLastError();
}

}  // namespace ctu
