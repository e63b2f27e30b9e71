// Deliberate defects, one per mode, run through the host emulation to show that
// its checks fire (test infrastructure; none of this is library code):
//   race     thread 0 rewrites a __shared__ value that other threads read with
//            no barrier between (ThreadSanitizer)
//   oob      a write one element past the dynamic LDS block (AddressSanitizer)
//   diverge  half the work-group waits at one barrier, half at another
//   stall    one thread skips a barrier the others wait at (barrier time-out)
//   clean    the race kernel with the missing barrier in place (no report)
#include <hip/hip_runtime.h>

#include <cstring>

__global__ void race_kernel(int* out, int fixed) {
  __shared__ int v;
  if (threadIdx.x == 0) v = 1;
  __syncthreads();
  int r = v;
  if (fixed) __syncthreads();
  if (threadIdx.x == 0) v = 2;
  __syncthreads();
  out[threadIdx.x] = r + v;
}

__global__ void oob_kernel(int n) {
  char* lds = ::emu::dyn_lds();
  if (threadIdx.x == 0) lds[n] = 1;
  __syncthreads();
}

__global__ void diverge_kernel(int) {
  if (threadIdx.x < 128) {
    __syncthreads();
  } else {
    __syncthreads();
  }
}

__global__ void stall_kernel(int) {
  if (threadIdx.x != 7) __syncthreads();
}

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  static int out[256];
  if (!strcmp(argv[1], "race") || !strcmp(argv[1], "clean")) {
    hipLaunchKernelGGL(race_kernel, dim3(1), dim3(256), 0, 0, out, (int)!strcmp(argv[1], "clean"));
  } else if (!strcmp(argv[1], "oob")) {
    hipLaunchKernelGGL(oob_kernel, dim3(1), dim3(64), 512, 0, 512);
  } else if (!strcmp(argv[1], "diverge")) {
    hipLaunchKernelGGL(diverge_kernel, dim3(1), dim3(256), 0, 0, 0);
  } else if (!strcmp(argv[1], "stall")) {
    hipLaunchKernelGGL(stall_kernel, dim3(1), dim3(64), 0, 0, 0);
  } else {
    return 2;
  }
  return 0;
}
