// Filter and discretisation kernels of one state layout (INST_B0, INST_B1),
// compiled once per layout.
#include "filter_kernel.h"

template int launch_filter_layout<INST_B0, INST_B1>(const DevModel &, bool, const FilterLaunch &, hipStream_t);
template int launch_discretize_layout<INST_B0, INST_B1>(const DevModel &, const double *, int64_t, double *,
                                                        double *, WsCtl *, hipStream_t);
