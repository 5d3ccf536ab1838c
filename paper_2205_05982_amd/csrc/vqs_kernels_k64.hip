// Kernel instantiations for 64-bit keys: the default level tile size and the kernels
// that do not depend on it.
#define VQS_BITS 64
#define VQS_LI level_chunks(64)
#define VQS_WITH_SOLO 1
#include "vqs_instantiate.inc"
