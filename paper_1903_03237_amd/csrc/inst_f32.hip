// Kernel instantiations for the P32 precision policy.
#define FM_P P32
#define FM_SUFFIX f32
#include "launch.inc"
