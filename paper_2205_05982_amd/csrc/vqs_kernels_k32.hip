// Kernel instantiations for 32-bit keys.
#define VQS_BITS 32
#include "vqs_instantiate.inc"
