// vqs_stable.hip -- packing kernels of the stable sort (see vqs_stable.h).
#include "vqs_device.h"
#include "vqs_stable.h"

namespace vqs {

namespace {

constexpr int ST_P = 256;

template <int BITS>
__global__ void __launch_bounds__(ST_P) pack_kernel(const typename Key<BITS>::S* keys, uint64_t n, int mode,
                                                     int comp, void* out) {
  using K = Key<BITS>;
  const uint64_t stride = (uint64_t)gridDim.x * ST_P;
  for (uint64_t i = (uint64_t)blockIdx.x * ST_P + threadIdx.x; i < n; i += stride) {
    const uint64_t k = (uint64_t)K::load_t(keys[i], mode);
    if (comp == COMP64) {
      static_cast<uint64_t*>(out)[i] = (k << 32) | i;
    } else {
      u128k c;
      c.lo = i;
      c.hi = k;
      static_cast<u128k*>(out)[i] = c;
    }
  }
}

template <int BITS>
__global__ void __launch_bounds__(ST_P) unpack_kernel(const void* comp_keys, uint64_t n, int mode, int comp,
                                                       typename Key<BITS>::S* keys, uint64_t* rows) {
  using K = Key<BITS>;
  using R = typename K::R;
  const uint64_t stride = (uint64_t)gridDim.x * ST_P;
  for (uint64_t i = (uint64_t)blockIdx.x * ST_P + threadIdx.x; i < n; i += stride) {
    uint64_t k, row;
    if (comp == COMP64) {
      const uint64_t c = static_cast<const uint64_t*>(comp_keys)[i];
      k = c >> 32;
      row = c & 0xFFFFFFFFull;
    } else {
      const u128k c = static_cast<const u128k*>(comp_keys)[i];
      k = c.hi;
      row = c.lo;
    }
    keys[i] = K::store_t((R)k, mode);
    if (rows) rows[i] = row;
  }
}

int grid_of(uint64_t n) {
  uint64_t g = (n + ST_P - 1) / ST_P;
  if (g > 8192) g = 8192;
  return g < 1 ? 1 : (int)g;
}

}  // namespace

hipError_t launch_stable_pack(const void* keys, uint64_t n, int bits, int mode, int comp, void* out,
                              hipStream_t s) {
  const int g = grid_of(n);
  switch (bits) {
    case 16:
      hipLaunchKernelGGL(pack_kernel<16>, dim3(g), dim3(ST_P), 0, s, (const uint16_t*)keys, n, mode, comp, out);
      break;
    case 32:
      hipLaunchKernelGGL(pack_kernel<32>, dim3(g), dim3(ST_P), 0, s, (const uint32_t*)keys, n, mode, comp, out);
      break;
    case 64:
      hipLaunchKernelGGL(pack_kernel<64>, dim3(g), dim3(ST_P), 0, s, (const uint64_t*)keys, n, mode, comp, out);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_stable_unpack(const void* comp_keys, uint64_t n, int bits, int mode, int comp, void* keys,
                                uint64_t* rows, hipStream_t s) {
  const int g = grid_of(n);
  switch (bits) {
    case 16:
      hipLaunchKernelGGL(unpack_kernel<16>, dim3(g), dim3(ST_P), 0, s, comp_keys, n, mode, comp, (uint16_t*)keys,
                         rows);
      break;
    case 32:
      hipLaunchKernelGGL(unpack_kernel<32>, dim3(g), dim3(ST_P), 0, s, comp_keys, n, mode, comp, (uint32_t*)keys,
                         rows);
      break;
    case 64:
      hipLaunchKernelGGL(unpack_kernel<64>, dim3(g), dim3(ST_P), 0, s, comp_keys, n, mode, comp, (uint64_t*)keys,
                         rows);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace vqs
