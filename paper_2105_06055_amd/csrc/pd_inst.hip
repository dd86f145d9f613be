// pd_inst.hip -- explicit instantiation of the per-dtype implementation
// (PD_INST_T = float or double; PD_INST_PART selects a share of it: 0 .. 3
// the entry-point implementations, 4 .. 6 the (y, z) pass kernels), so that
// the library's device code compiles in parallel units.
#include "pd_impl.hpp"

#ifndef PD_INST_T
#error "PD_INST_T must be defined (float or double)"
#endif
#ifndef PD_INST_PART
#error "PD_INST_PART must be defined (0 .. 6)"
#endif

namespace pdi {
#if PD_INST_PART == 0
template pd_status force_impl<PD_INST_T>(pd_plan, const PD_INST_T*, const void*, PD_INST_T*, PD_INST_T*, hipStream_t);
#elif PD_INST_PART == 1
template pd_status verlet_impl<PD_INST_T>(pd_plan, pd_state*, const PD_INST_T*, const PD_INST_T*, double, int, double*,
                                          hipStream_t);
#elif PD_INST_PART == 2
template pd_status verlet_adjoint_impl<PD_INST_T>(pd_plan, const PD_INST_T*, const PD_INST_T*, const PD_INST_T*,
                                                  PD_INST_T*, PD_INST_T*, PD_INST_T*, PD_INST_T*, double, hipStream_t);
template pd_status cg_run<PD_INST_T, PD_INST_T>(pd_plan, PD_INST_T*, PD_INST_T*, PD_INST_T*, PD_INST_T*, PD_INST_T*,
                                                double, double, int, int*, int*, double*, hipStream_t);
template pd_status lin_apply<PD_INST_T, 3>(pd_plan, const PD_INST_T*, PD_INST_T*, const PD_INST_T*, hipStream_t);
template pd_status lin_apply<PD_INST_T, 2>(pd_plan, const PD_INST_T*, PD_INST_T*, const PD_INST_T*, hipStream_t);
template pd_status precond_apply<PD_INST_T, double, PD_INST_T>(pd_plan, const double*, PD_INST_T*, hipStream_t);
#if PD_INST_F32
template pd_status precond_apply<float, float, float>(pd_plan, const float*, float*, hipStream_t);
#endif
#elif PD_INST_PART == 4
#define PD_YZ_DEF(T, M) template pd_status launch_yzconv<T, M>(pd_plan, const M&, int, int, hipStream_t);
PD_YZ_LIST_A(PD_YZ_DEF, PD_INST_T)
#elif PD_INST_PART == 5
#define PD_YZ_DEF(T, M) template pd_status launch_yzconv<T, M>(pd_plan, const M&, int, int, hipStream_t);
PD_YZ_LIST_B(PD_YZ_DEF, PD_INST_T)
#elif PD_INST_PART == 6
template pd_status nbb_yz<PD_INST_T>(pd_plan, int, hipStream_t);
#else
template pd_status plan_alloc<PD_INST_T>(pd_plan, hipStream_t, const uint8_t*, const uint8_t*);
template pd_status build_device_tables<PD_INST_T>(pd_plan, const std::vector<Bond>&, hipStream_t);
template pd_status adjoint_impl<PD_INST_T>(pd_plan, const PD_INST_T*, const PD_INST_T*, const void*, const PD_INST_T*,
                                           PD_INST_T*, PD_INST_T*, PD_INST_T, int, hipStream_t);
template pd_status damage_impl<PD_INST_T>(pd_plan, const uint8_t*, PD_INST_T*, hipStream_t);
template pd_status test_conv_impl<PD_INST_T>(pd_plan, const PD_INST_T*, const int*, int, PD_INST_T*, hipStream_t);
#endif
}  // namespace pdi
