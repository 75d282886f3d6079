// Plain FP64 baseline scan of one state layout (INST_B0, INST_B1), compiled
// once per layout.
#include "plain_kernel.h"

template int launch_plain_layout<INST_B0, INST_B1>(const DevModel &, const PlainLaunch &, hipStream_t);
