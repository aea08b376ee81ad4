// probe.hpp - bandwidth references for the roofline of the step (included
// by lbm.hip inside its anonymous namespace).  Not part of the method: they
// calibrate what HBM delivers to plain streaming kernels on this device.
//
//  k_copy16   one 16-byte vector per thread, one-shot grid: the plain copy
//             (optionally with non-temporal loads and stores).
//  k_rows     the step's streaming pattern without its arithmetic: every
//             thread reads 8 bytes from each of R rows (row_stride bytes
//             apart, the same offset in each) and writes them to the same
//             places of the destination, all loads before the stores.

template <bool NT>
__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ a, float4* __restrict__ b,
                                                size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if constexpr (NT) {
    float4 v;
    v.x = __builtin_nontemporal_load(&a[i].x);
    v.y = __builtin_nontemporal_load(&a[i].y);
    v.z = __builtin_nontemporal_load(&a[i].z);
    v.w = __builtin_nontemporal_load(&a[i].w);
    __builtin_nontemporal_store(v.x, &b[i].x);
    __builtin_nontemporal_store(v.y, &b[i].y);
    __builtin_nontemporal_store(v.z, &b[i].z);
    __builtin_nontemporal_store(v.w, &b[i].w);
  } else {
    b[i] = a[i];
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_rows(const char* __restrict__ a, char* __restrict__ b,
                                              size_t row_stride, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float2 v[R];
#pragma unroll
  for (int l = 0; l < R; ++l) v[l] = *(const float2*)(a + (size_t)l * row_stride + i * 8);
#pragma unroll
  for (int l = 0; l < R; ++l) *(float2*)(b + (size_t)l * row_stride + i * 8) = v[l];
}
