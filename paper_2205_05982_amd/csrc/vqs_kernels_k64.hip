// Kernel instantiations for 64-bit keys.
#define VQS_BITS 64
#include "vqs_instantiate.inc"
