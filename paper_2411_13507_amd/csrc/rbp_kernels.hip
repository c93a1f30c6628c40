// Batched segment-QP kernels for gfx950, default launch shape: one 64-lane
// wavefront (one instance) per workgroup, one launch per (degree,
// reachable-row class) group of the work order.  The device code is in
// rbp_segment.hpp; the other launch shapes are in rbp_kernels_var.hip.
#include "rbp_segment.hpp"

namespace rbp {
namespace {

// One launch per degree P: block b solves order[inst_base + b]; instances
// are grouped by degree in the work order.
template <typename Real, int P, bool kAdmm>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void solve_kernel(SolveArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int b = blockIdx.x + A.inst_base;
  if (b >= A.N) return;
  const InstDesc dsc = A.desc[b];
  if (dsc.p == P) solve_instance<P, Real, kAdmm>(A, dsc, smem);
  else if (threadIdx.x == 0) { A.status_out[dsc.inst] = kInvalid; if (A.store) A.fw_status[dsc.inst] = kInvalid; }
}

// One launch per group of the work order (same degree P): block b handles
// order[inst_base + b].
template <int P>
__global__ __launch_bounds__(64) void backward_kernel(BackArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int b = blockIdx.x + A.inst_base;
  if (b >= A.N) return;
  const InstDesc dsc = A.desc[b];
  if (dsc.p == P) backward_instance<P>(A, dsc, smem);
}

}  // namespace

LdsDims make_dims(int pmax, int r_cap, int nf_cap, int real_bytes, bool admm) {
  LdsDims d{};
  d.nmax = 3 * (pmax - 1);
  d.ncol = 3 * (pmax + 1);
  d.r_cap = r_cap < 1 ? 1 : r_cap;
  d.nf_cap = nf_cap < 1 ? 1 : nf_cap;
  d.m_cap = (pmax - 1) * d.nf_cap + 6 * pmax - 3 + d.r_cap;
  int o = 0;
  auto take = [&](int bytes) { const int at = o; o += (bytes + 15) & ~15; return at; };
  d.o_Hd = take(d.r_cap * (d.ncol | 1) * 8);
  d.o_Af = take(d.nf_cap * 3 * 8);
  d.o_rowval = take(d.m_cap * 8);
  d.o_ybuf = take(2 * d.ncol * 8);
  d.o_vec = take(5 * d.nmax * 8);   // vA..vE
  d.o_scal = take(16 * 8);
  d.o_acte = take(2 * d.nmax * 8);
  d.o_lam = take(d.nmax * 8);
  d.o_actid = take(d.nmax * 4);
  d.o_actside = take(d.nmax * 4);
  d.o_cst = take(((admm ? 2 : 1) * kMaxFree * kMaxFree + kMaxPts * kMaxPts) * 8);
  d.o_Rd = take(d.nmax * 8);
  d.o_region = o;
  // iteration scratch in the precision of the iterations
  const int hs = d.r_cap | 1;
  const int rb = real_bytes;
  int a = d.o_region;
  auto take_r = [&](int bytes) { const int at = a; a += (bytes + 15) & ~15; return at; };
  if (admm) {
    d.o_Hf = take_r(d.nmax * hs * rb);
    d.o_Aff = take_r(d.nf_cap * 4 * rb);
    d.o_vbuf = take_r(d.m_cap * rb);
    d.o_xb1 = take_r(d.nmax * rb);
    d.o_xb2 = take_r(d.nmax * rb);
    d.o_Kx = take_r(d.nmax * d.nmax * rb);
  } else {
    d.o_Hf = d.o_Aff = d.o_vbuf = d.o_xb1 = d.o_xb2 = d.o_Kx = d.o_region;   // unused
  }
  int b = d.o_region;
  auto take_p = [&](int bytes) { const int at = b; b += (bytes + 15) & ~15; return at; };
  d.o_Q1 = take_p(d.nmax * (d.nmax | 1) * 8);
  d.o_R = take_p(d.nmax * (d.nmax | 1) * 8);
  d.o_Ri = take_p(d.nmax * (d.nmax | 1) * 8);
  d.bytes = a > b ? a : b;
  return d;
}

// The backward pass reads the faces, the factor of the final working set,
// its ids, sides and multipliers, the coefficients of its reachable rows on
// the pinned points (six per active row, packed by working-set slot in the
// Hd region), the degree table L^-1 and a few vectors; everything else of the
// forward carve aliases the start of the buffer and is never touched.
LdsDims make_back_dims(int pmax, int nf_cap) {
  LdsDims d{};
  d.nmax = 3 * (pmax - 1);
  d.ncol = 3 * (pmax + 1);
  d.r_cap = 1;
  d.nf_cap = nf_cap < 1 ? 1 : nf_cap;
  d.m_cap = 1;
  int o = 0;
  auto take = [&](int bytes) { const int at = o; o += (bytes + 15) & ~15; return at; };
  d.o_Hd = take(d.nmax * 6 * 8);
  d.o_Af = take(d.nf_cap * 3 * 8);
  d.o_ybuf = take(2 * d.ncol * 8);
  d.o_vec = take(5 * d.nmax * 8);
  d.o_scal = take(16 * 8);
  d.o_lam = take(d.nmax * 8);
  d.o_actid = take(d.nmax * 4);
  d.o_actside = take(d.nmax * 4);
  d.o_cst = take(kMaxFree * kMaxFree * 8);
  d.o_Q1 = take(d.nmax * (d.nmax | 1) * 8);
  d.o_R = take(d.nmax * (d.nmax | 1) * 8);
  d.o_rowval = d.o_acte = d.o_Rd = d.o_Ri = 0;
  d.o_region = d.o_Hf = d.o_Aff = d.o_vbuf = d.o_xb1 = d.o_xb2 = d.o_Kx = 0;
  d.bytes = o;
  return d;
}

hipError_t upload_constants(int device) {
  (void)device;
  DegConst host[kMaxDeg + 1];
  std::memset(host, 0, sizeof(host));
  for (int p = kMinDeg; p <= kMaxDeg; ++p)
    if (!build_degree(p, host[p])) return hipErrorInvalidValue;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_deg), host, sizeof(host), 0, hipMemcpyHostToDevice);
}

template <typename Real, bool kAdmm>
static void launch_solve_t(const SolveArgs& a, int n_blocks, hipStream_t s, int pfix) {
  const dim3 g(n_blocks), blk(kWave);
  const size_t sh = a.dims.bytes;
  switch (pfix) {
    case 3: hipLaunchKernelGGL((solve_kernel<Real, 3, kAdmm>), g, blk, sh, s, a); break;
    case 4: hipLaunchKernelGGL((solve_kernel<Real, 4, kAdmm>), g, blk, sh, s, a); break;
    case 5: hipLaunchKernelGGL((solve_kernel<Real, 5, kAdmm>), g, blk, sh, s, a); break;
    case 6: hipLaunchKernelGGL((solve_kernel<Real, 6, kAdmm>), g, blk, sh, s, a); break;
    case 7: hipLaunchKernelGGL((solve_kernel<Real, 7, kAdmm>), g, blk, sh, s, a); break;
    case 8: hipLaunchKernelGGL((solve_kernel<Real, 8, kAdmm>), g, blk, sh, s, a); break;
    case 9: hipLaunchKernelGGL((solve_kernel<Real, 9, kAdmm>), g, blk, sh, s, a); break;
    default: break;
  }
}

// polish only (no ADMM iterations): one variant, its iteration precision is
// irrelevant; otherwise FP32 or FP64 iterations
hipError_t launch_solve(const SolveArgs& a, int n_blocks, hipStream_t s, bool fp64_iters, int pfix) {
  if (n_blocks <= 0) return hipSuccess;
  if (a.admm_iters == 0) launch_solve_t<float, false>(a, n_blocks, s, pfix);
  else if (fp64_iters) launch_solve_t<double, true>(a, n_blocks, s, pfix);
  else launch_solve_t<float, true>(a, n_blocks, s, pfix);
  return hipGetLastError();
}

hipError_t launch_backward(const BackArgs& a, int n_blocks, hipStream_t s, int pfix) {
  if (n_blocks <= 0) return hipSuccess;
  const dim3 g(n_blocks), blk(kWave);
  const size_t sh = a.dims.bytes;
  switch (pfix) {
    case 3: hipLaunchKernelGGL((backward_kernel<3>), g, blk, sh, s, a); break;
    case 4: hipLaunchKernelGGL((backward_kernel<4>), g, blk, sh, s, a); break;
    case 5: hipLaunchKernelGGL((backward_kernel<5>), g, blk, sh, s, a); break;
    case 6: hipLaunchKernelGGL((backward_kernel<6>), g, blk, sh, s, a); break;
    case 7: hipLaunchKernelGGL((backward_kernel<7>), g, blk, sh, s, a); break;
    case 8: hipLaunchKernelGGL((backward_kernel<8>), g, blk, sh, s, a); break;
    case 9: hipLaunchKernelGGL((backward_kernel<9>), g, blk, sh, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rbp

