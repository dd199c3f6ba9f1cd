// LDS read bandwidth probe (measurement helper, not part of the library):
// every workgroup streams 16-byte reads from its 16 KiB of LDS, four in
// flight per wavefront, and the host times the launch with HIP events.
// Built by lds_bandwidth.py.
#include <hip/hip_runtime.h>

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeWords = 1024;  // uint4 words: 16 KiB of LDS per workgroup

__global__ __launch_bounds__(kProbeThreads) void k_lds_read(unsigned int *out, int iters)
{
    __shared__ uint4 buf[kProbeWords];
    for (int i = threadIdx.x; i < kProbeWords; i += kProbeThreads)
        buf[i] = make_uint4(i, 3u * i, 5u * i, 7u * i);
    __syncthreads();
    unsigned int acc = 0;
    int idx = threadIdx.x;
    for (int it = 0; it < iters; it += 4) {
        // consecutive lanes read consecutive 16-byte words: no bank conflicts
        const uint4 v0 = buf[idx];
        const uint4 v1 = buf[(idx + kProbeThreads) & (kProbeWords - 1)];
        const uint4 v2 = buf[(idx + 2 * kProbeThreads) & (kProbeWords - 1)];
        const uint4 v3 = buf[(idx + 3 * kProbeThreads) & (kProbeWords - 1)];
        // all 16 words enter the result through three-input XORs (two
        // instructions per read), so the vector ALU stays far from the bound
        acc = __builtin_amdgcn_bitop3_b32(acc, __builtin_amdgcn_bitop3_b32(v0.x, v0.y, v0.z, 0x96), v0.w, 0x96);
        acc = __builtin_amdgcn_bitop3_b32(acc, __builtin_amdgcn_bitop3_b32(v1.x, v1.y, v1.z, 0x96), v1.w, 0x96);
        acc = __builtin_amdgcn_bitop3_b32(acc, __builtin_amdgcn_bitop3_b32(v2.x, v2.y, v2.z, 0x96), v2.w, 0x96);
        acc = __builtin_amdgcn_bitop3_b32(acc, __builtin_amdgcn_bitop3_b32(v3.x, v3.y, v3.z, 0x96), v3.w, 0x96);
        idx = (idx + 16) & (kProbeWords - 1);
        __asm__ volatile("" ::: "memory");  // the next group's reads are not merged with these
    }
    if (acc == 0x9E3779B9u) out[blockIdx.x] = acc;  // keeps the reads alive
}

}  // namespace

// Times `reps` launches of `blocks` workgroups reading 16 * iters bytes per
// thread; returns 0 and the mean milliseconds per launch, or a HIP error code.
extern "C" int lds_probe_run(int blocks, int iters, int reps, double *ms_per_launch)
{
    unsigned int *out = nullptr;
    hipError_t e = hipMalloc((void **)&out, sizeof(unsigned int) * (size_t)blocks);
    if (e != hipSuccess) return (int)e;
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(kProbeThreads), 0, 0, out, iters);  // warm-up
    (void)hipEventRecord(t0, 0);
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(kProbeThreads), 0, 0, out, iters);
    (void)hipEventRecord(t1, 0);
    e = hipEventSynchronize(t1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    *ms_per_launch = (double)ms / reps;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(out);
    return e == hipSuccess ? (int)hipGetLastError() : (int)e;
}
