// The persistent step (one launch per step, SBT_OPT_PERSISTENT) as a module
// of its own: the kernels' source compiled with SBT_PERSISTENT_TU keeps only
// the persistent kernel and its launchers.  Kept apart, the plan-builder and
// forcing-loop kernels of the main module address their LDS as they do
// without it.
#define SBT_PERSISTENT_TU 1
#include "sbt_kernels.hip"
