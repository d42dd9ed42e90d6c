#include <hip/hip_runtime.h>
__global__ void k(const float4 *g, float4 *out) {
    __shared__ float4 s[256];
    const int t = threadIdx.x;
    __builtin_amdgcn_global_load_lds((const void *)(g + t), (__attribute__((address_space(3))) void *)(s + (t & ~63)), 16, 0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    out[t] = s[255 - t];
}
