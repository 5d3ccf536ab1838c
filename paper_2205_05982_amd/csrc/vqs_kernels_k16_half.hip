// Kernel instantiations for 16-bit keys: the level kernels with half-size tiles.
#define VQS_BITS 16
#define VQS_LI level_chunks_half(16)
#define VQS_WITH_SOLO 0
#include "vqs_instantiate.inc"
