// Smoother kernels of one state layout (INST_B0, INST_B1), compiled once per
// layout.
#include "smoother_kernel.h"

template int launch_smoother_layout<INST_B0, INST_B1>(const DevModel &, bool, const SmoothLaunch &, hipStream_t);
