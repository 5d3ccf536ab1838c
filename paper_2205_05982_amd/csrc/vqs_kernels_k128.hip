// Kernel instantiations for 128-bit keys.
#define VQS_BITS 128
#include "vqs_instantiate.inc"
