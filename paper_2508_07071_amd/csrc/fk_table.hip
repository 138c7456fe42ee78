// Run-table upload (Section IV-B: the batch's per-item parameters reach the
// device before the fused kernel reads them).  A kernel on the run's own
// stream copies the table from the pinned host staging buffer into device
// memory, so the fused kernel after it waits on a kernel of the same queue
// rather than on a copy engine's completion signal.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fk {

// 16-byte units [0, n0) and [off1, off1 + n1) of src are copied to the same
// offsets of dst; one unit per lane.
__global__ void __launch_bounds__(256) k_table_upload(const uint4 *__restrict__ src,
                                                      uint4 *__restrict__ dst, uint32_t n0,
                                                      uint32_t off1, uint32_t n1)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n0) {
        dst[i] = src[i];
    } else if (i - n0 < n1) {
        const uint32_t j = off1 + (i - n0);
        dst[j] = src[j];
    }
}

const void *kernel_table_upload()
{
    return (const void *)k_table_upload;
}

}  // namespace fk
