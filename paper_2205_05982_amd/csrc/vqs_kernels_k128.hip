// Kernel instantiations for 128-bit keys: the default level tile size and the kernels
// that do not depend on it.
#define VQS_BITS 128
#define VQS_LI level_chunks(128)
#define VQS_WITH_SOLO 1
#include "vqs_instantiate.inc"
