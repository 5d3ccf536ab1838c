// Kernel instantiations for 16-bit keys.
#define VQS_BITS 16
#include "vqs_instantiate.inc"
