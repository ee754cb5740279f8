// Descriptor-table setup and state copy kernels of the batched step.
#include "rd_batch.h"

namespace rd {

// Thread i copies descriptor i of this chunk into the device table.
__global__ void batch_setup_kernel(BatchSetupArgs a) {
  const int i = threadIdx.x;
  if (i < a.count) a.table[a.first + i] = a.inst[i];
}

// b <- a for every array of every instance; blockIdx.y = instance.
__global__ void batch_copy_kernel(BatchCopyArgs a) {
  const BatchInst& I = a.table[blockIdx.y];
  const size_t cells = (size_t)I.nx * (size_t)I.ny;
  const size_t total = cells * (size_t)a.nf;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x) {
    const size_t f = k / cells, o = k - f * cells;
    I.b[f][o] = I.a[f][o];
  }
}

}  // namespace rd
