// Test helper only: Philox4x32-10 blocks from rocRAND's device generator, to
// cross-check the library's own Philox (a second, independent
// implementation).  Not part of the library; the tests load it with ctypes.
//
// rocRAND's philox state is (seed, subsequence, offset): the key is the
// seed, the 128-bit counter's upper half the subsequence and its lower half
// offset / 4, so the block of counter (c0, c1, c2, c3) is the first rocrand4()
// of rocrand_init(seed, c2 + 2^32 c3, 4 (c0 + 2^32 c1)).  The test checks
// that reading by comparing with the library's words.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>

#include <cstdint>

__global__ void k_rocrand_blocks(uint64_t seed, const uint4 *ctr, uint32_t m, uint4 *out)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint4 c = ctr[j];
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, (uint64_t)c.z | ((uint64_t)c.w << 32),
                 4ull * ((uint64_t)c.x | ((uint64_t)c.y << 32)), &st);
    out[j] = rocrand4(&st);
}

// ctr: host [4 m] counters; out: host [4 m] blocks.  Returns a hipError_t.
extern "C" int rocrand_philox_blocks(uint64_t seed, const uint32_t *ctr, uint32_t m, uint32_t *out)
{
    if (m == 0) return 0;
    uint4 *dc = nullptr, *dout = nullptr;
    hipError_t e = hipMalloc(&dc, sizeof(uint4) * m);
    if (e == hipSuccess) e = hipMalloc(&dout, sizeof(uint4) * m);
    if (e == hipSuccess) e = hipMemcpy(dc, ctr, sizeof(uint4) * m, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_rocrand_blocks, dim3((m + 255) / 256), dim3(256), 0, 0, seed, dc, m, dout);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, sizeof(uint4) * m, hipMemcpyDeviceToHost);
    hipFree(dc);
    hipFree(dout);
    return (int)e;
}
