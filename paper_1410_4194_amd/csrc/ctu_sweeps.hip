// ctu_sweeps.hip -- instantiates the sweep kernels for one storage type, solver class and
// reconstruction.  The build compiles this file once per (CTU_SWEEP_T, CTU_SWEEP_K,
// CTU_SWEEP_R) triple, in parallel: double and float; the exact solver for K = 0 (any
// gamma), 3 (gamma = 5/3) and 5 (gamma = 7/5), the Roe solver (K = kRoe = 1) and Roe with the
// H correction (K = kRoeH = 2); PPMC (R = 0) and PPMP (R = 1).
#include "ctu_sweeps.hpp"

#if !defined(CTU_SWEEP_T) || !defined(CTU_SWEEP_K) || !defined(CTU_SWEEP_R)
#error "compile with -DCTU_SWEEP_T=<double|float> -DCTU_SWEEP_K=<0|1|2|3|5> -DCTU_SWEEP_R=<0|1>"
#endif

namespace ctu {

template <>
hipError_t launch_sweeps<CTU_SWEEP_T, CTU_SWEEP_K, CTU_SWEEP_R>(const PlanView& v, int stage,
                                                                hipStream_t stream,
                                                                Profiler* prof) {
  // the Newton histogram exists for the exact solver only
  if constexpr (CTU_SWEEP_K != kRoe && CTU_SWEEP_K != kRoeH) {
    if (prof && prof->hist)
      return enqueue_sweeps<CTU_SWEEP_T, CTU_SWEEP_K, true, CTU_SWEEP_R>(v, stage, stream, prof);
  }
  return enqueue_sweeps<CTU_SWEEP_T, CTU_SWEEP_K, false, CTU_SWEEP_R>(v, stage, stream, prof);
}

}  // namespace ctu
