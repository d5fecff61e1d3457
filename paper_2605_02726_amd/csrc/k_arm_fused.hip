// ARM entropy model, fused BF16 MFMA form (placeholder until the MFMA kernel
// lands: reports the shape as unsupported so the plain kernel runs).
#include "cc_internal.h"

int cc_arm_fused_supported(const DevDesc&) { return 0; }
int cc_launch_arm_fused(const Launch&, const DevDesc&, int, hipStream_t) { return CC_EINVAL; }
