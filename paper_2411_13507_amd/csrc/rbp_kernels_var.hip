// Batched segment-QP kernels for gfx950, the launch shapes other than the
// default (rbp_kernels.hip) and the single-launch schedule; device code in
// rbp_segment.hpp.  These kernels are separate instantiations in their own
// translation unit, so that adding them leaves the code of the default
// kernels unchanged (a device function with several callers may be compiled
// out of line).
#include "rbp_segment.hpp"

namespace rbp {
namespace {

// Grouped schedule with WPG wavefronts (instances) per workgroup: wave w of
// block b solves order[inst_base + WPG b + w] in its own slice of the
// block's LDS; WPE is the number of wavefronts per SIMD the register budget
// is sized for.
template <int P, bool kAdmm, int WPG, int WPE>
__global__ __launch_bounds__(64 * WPG) __attribute__((amdgpu_waves_per_eu(WPE))) void solve_kernel_shape(SolveArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int w = threadIdx.x >> 6;
  const int b = blockIdx.x * WPG + w + A.inst_base;
  if (b >= A.N) return;
  const InstDesc dsc = A.desc[b];
  // (one wavefront: the LDS base stays a constant)
  char* my = WPG == 1 ? smem : smem + size_t(w) * size_t(A.dims.bytes);
  if (dsc.p == P) solve_instance<P, float, kAdmm, (WPG > 1), 10 * WPG + WPE>(A, dsc, my);
  else if ((threadIdx.x & (kWave - 1)) == 0) { A.status_out[dsc.inst] = kInvalid; if (A.store) A.fw_status[dsc.inst] = kInvalid; }
}

// The whole batch in one launch: block b solves order[b] whatever its degree
// (the degree picks the instantiation inside the kernel), LDS sized for the
// batch's largest instance.
template <bool kAdmm>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void solve_kernel_all(SolveArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int b = blockIdx.x + A.inst_base;
  if (b >= A.N) return;
  const InstDesc dsc = A.desc[b];
  switch (dsc.p) {
    case 3: solve_instance<3, float, kAdmm, false, 99>(A, dsc, smem); break;
    case 4: solve_instance<4, float, kAdmm, false, 99>(A, dsc, smem); break;
    case 5: solve_instance<5, float, kAdmm, false, 99>(A, dsc, smem); break;
    case 6: solve_instance<6, float, kAdmm, false, 99>(A, dsc, smem); break;
    case 7: solve_instance<7, float, kAdmm, false, 99>(A, dsc, smem); break;
    case 8: solve_instance<8, float, kAdmm, false, 99>(A, dsc, smem); break;
    case 9: solve_instance<9, float, kAdmm, false, 99>(A, dsc, smem); break;
    default: if (threadIdx.x == 0) { A.status_out[dsc.inst] = kInvalid; if (A.store) A.fw_status[dsc.inst] = kInvalid; } break;
  }
}

// Backward pass of a single-launch forward: the whole batch in one launch.
__global__ __launch_bounds__(64) void backward_kernel_all(BackArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int b = blockIdx.x + A.inst_base;
  if (b >= A.N) return;
  const InstDesc dsc = A.desc[b];
  switch (dsc.p) {
    case 3: backward_instance<3>(A, dsc, smem); break;
    case 4: backward_instance<4>(A, dsc, smem); break;
    case 5: backward_instance<5>(A, dsc, smem); break;
    case 6: backward_instance<6>(A, dsc, smem); break;
    case 7: backward_instance<7>(A, dsc, smem); break;
    case 8: backward_instance<8>(A, dsc, smem); break;
    case 9: backward_instance<9>(A, dsc, smem); break;
    default: break;
  }
}

template <bool kAdmm, int WPG, int WPE>
void launch_shape_t(const SolveArgs& a, int n_inst, hipStream_t s, int pfix) {
  const dim3 g((n_inst + WPG - 1) / WPG), blk(kWave * WPG);
  const size_t sh = size_t(a.dims.bytes) * WPG;
  switch (pfix) {
    case 3: hipLaunchKernelGGL((solve_kernel_shape<3, kAdmm, WPG, WPE>), g, blk, sh, s, a); break;
    case 4: hipLaunchKernelGGL((solve_kernel_shape<4, kAdmm, WPG, WPE>), g, blk, sh, s, a); break;
    case 5: hipLaunchKernelGGL((solve_kernel_shape<5, kAdmm, WPG, WPE>), g, blk, sh, s, a); break;
    case 6: hipLaunchKernelGGL((solve_kernel_shape<6, kAdmm, WPG, WPE>), g, blk, sh, s, a); break;
    case 7: hipLaunchKernelGGL((solve_kernel_shape<7, kAdmm, WPG, WPE>), g, blk, sh, s, a); break;
    case 8: hipLaunchKernelGGL((solve_kernel_shape<8, kAdmm, WPG, WPE>), g, blk, sh, s, a); break;
    case 9: hipLaunchKernelGGL((solve_kernel_shape<9, kAdmm, WPG, WPE>), g, blk, sh, s, a); break;
    default: break;
  }
}

template <bool kAdmm>
void launch_shape_k(const SolveArgs& a, int n_inst, hipStream_t s, int pfix, int shape) {
  if (shape == kShapeW1E1) launch_shape_t<kAdmm, 1, 1>(a, n_inst, s, pfix);
  else launch_shape_t<kAdmm, 2, 2>(a, n_inst, s, pfix);
}

}  // namespace

hipError_t upload_constants_var(int device) {
  (void)device;
  DegConst host[kMaxDeg + 1];
  std::memset(host, 0, sizeof(host));
  for (int p = kMinDeg; p <= kMaxDeg; ++p)
    if (!build_degree(p, host[p])) return hipErrorInvalidValue;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_deg), host, sizeof(host), 0, hipMemcpyHostToDevice);
}

hipError_t launch_solve_shape(const SolveArgs& a, int n_inst, hipStream_t s, int pfix, int shape) {
  if (n_inst <= 0) return hipSuccess;
  if (shape != kShapeW1E1 && shape != kShapeW2E2) return hipErrorInvalidValue;
  if (a.admm_iters == 0) launch_shape_k<false>(a, n_inst, s, pfix, shape);
  else launch_shape_k<true>(a, n_inst, s, pfix, shape);
  return hipGetLastError();
}

hipError_t launch_solve_all(const SolveArgs& a, int n_inst, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  const size_t sh = size_t(a.dims.bytes);
  if (a.admm_iters == 0) hipLaunchKernelGGL(solve_kernel_all<false>, dim3(n_inst), dim3(kWave), sh, s, a);
  else hipLaunchKernelGGL(solve_kernel_all<true>, dim3(n_inst), dim3(kWave), sh, s, a);
  return hipGetLastError();
}

hipError_t launch_backward_all(const BackArgs& a, int n_inst, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(backward_kernel_all, dim3(n_inst), dim3(kWave), size_t(a.dims.bytes), s, a);
  return hipGetLastError();
}

}  // namespace rbp
