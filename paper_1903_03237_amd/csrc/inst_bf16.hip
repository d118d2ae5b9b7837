// Kernel instantiations for the PBF precision policy.
#define FM_P PBF
#define FM_SUFFIX bf16
#include "launch.inc"
