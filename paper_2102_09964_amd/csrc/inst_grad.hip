// Log-likelihood adjoint kernels of one state layout (INST_B0, INST_B1),
// compiled once per layout.
#include "grad_kernel.h"

template int launch_grad_layout<INST_B0, INST_B1>(const DevModel &, bool, const GradLaunch &, hipStream_t);
