// Building the graph of Bezier curves (Sec. III-A, Thm. 2) and the adjacent
// hyperplanes of its nodes (Alg. 2, Sec. III-D).
//
// Edge i -> j when F [v_i; v_j] <= G, i.e. max_k (A_ik + B_jk) <= 0 with the
// per-node row values A = F1 v (start columns) and B = F2 v - G (end
// columns): an all-pairs (max, +) product of two N x m matrices followed by a
// sign test.  The pair kernel tiles it 64 x 64 with 4 x 4 register blocks and
// 16-row chunks of A and B staged in LDS (odd row stride), in FP64.  A tile
// is skipped with an exact bound: if min_i A_ik + min_j B_jk > 0 for some row
// k, every pair of the tile violates row k.  With nodes numbered along a
// space-filling curve most far-apart tiles go this way, so the work follows
// the number of near pairs rather than N^2; the result never depends on it.
// Output: the adjacency as a row-major bitmask (bit j % 32 of word j / 32 of
// row i) and out-degrees.
//
// Adjacent hyperplanes: per node, the nearest axis-aligned box (Euclidean
// distance, lowest index on ties), the closest point on it (a clamp) and the
// plane through that point with unit normal toward the node.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "rbp_internal.hpp"

namespace rbp {

// Workspace of the allocation-free graph run (rows A and B, tile minima):
// a fixed array in device memory, one copy per GPU, held until the process
// ends.  Host code never uses the name itself as an address: the device
// address of each GPU's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kGraphScratchDoubles];

namespace {

constexpr int kTile = 64;       // nodes per tile side
constexpr int kChunk = 16;      // rows of A, B per LDS stage
constexpr int kLd = kChunk + 1; // odd LDS stride in doubles
constexpr double kPad = -1e300; // rows beyond m: A + B stays far below 0

__global__ void graph_rows_kernel(GraphArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)a.n_nodes * a.m) return;
  const int i = (int)(t / a.m), k = (int)(t - (int64_t)i * a.m);
  double s1 = 0.0, s2 = 0.0;
  for (int c = 0; c < a.dim; ++c) {
    const double v = a.V[(int64_t)i * a.dim + c];
    s1 += a.F1[k * a.dim + c] * v;
    s2 += a.F2[k * a.dim + c] * v;
  }
  a.A[t] = s1;
  a.B[t] = s2 - a.G[k];
}

// per tile t and row k: minimum of A and of B over the tile's nodes
__global__ void graph_bounds_kernel(GraphArgs a, int n_tiles) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles * a.m) return;
  const int tile = t / a.m, k = t - tile * a.m;
  const int i0 = tile * kTile, i1 = i0 + kTile < a.n_nodes ? i0 + kTile : a.n_nodes;
  double ma = __builtin_huge_val(), mb = __builtin_huge_val();
  for (int i = i0; i < i1; ++i) {
    ma = fmin(ma, a.A[(int64_t)i * a.m + k]);
    mb = fmin(mb, a.B[(int64_t)i * a.m + k]);
  }
  a.Amin[t] = ma;
  a.Bmin[t] = mb;
}

__global__ __launch_bounds__(256) void graph_pairs_kernel(GraphArgs a) {
  __shared__ double As[kTile * kLd];
  __shared__ double Bs[kTile * kLd];
  __shared__ uint32_t words[kTile * 2];
  const int ti = blockIdx.y, tj = blockIdx.x;
  const int tid = threadIdx.x;
  const int n_words = (a.n_nodes + 31) / 32;
  // exact cull: a row violated by every pair of the tile
  bool culled = false;
  for (int k = 0; k < a.m && !culled; ++k) culled = a.Amin[ti * a.m + k] + a.Bmin[tj * a.m + k] > 0.0;
  if (tid < 2 * kTile) words[tid] = 0u;
  if (!culled) {
    const int r0 = (tid >> 4) * 4, c0 = (tid & 15) * 4;   // 4 x 4 block of the tile
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = -__builtin_huge_val();
    for (int k0 = 0; k0 < a.m; k0 += kChunk) {
      __syncthreads();
      // stage rows k0..k0+15 of the tile's A (start nodes) and B (end nodes)
      for (int e = tid; e < kTile * kChunk; e += 256) {
        const int n = e / kChunk, kk = e - n * kChunk, k = k0 + kk;
        const int gi = ti * kTile + n, gj = tj * kTile + n;
        As[n * kLd + kk] = (gi < a.n_nodes && k < a.m) ? a.A[(int64_t)gi * a.m + k] : kPad;
        Bs[n * kLd + kk] = (gj < a.n_nodes && k < a.m) ? a.B[(int64_t)gj * a.m + k] : kPad;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < kChunk; ++kk) {
        double av[4], bv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) av[r] = As[(r0 + r) * kLd + kk];
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[c] = Bs[(c0 + c) * kLd + kk];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[r][c] = fmax(acc[r][c], av[r] + bv[c]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = ti * kTile + r0 + r;
      uint32_t nib = 0u;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int gj = tj * kTile + c0 + c;
        if (acc[r][c] <= 0.0 && gi != gj && gi < a.n_nodes && gj < a.n_nodes) nib |= 1u << c;
      }
      if (nib) atomicOr(&words[(r0 + r) * 2 + (c0 >> 5)], nib << (c0 & 31));
    }
  }
  __syncthreads();
  if (tid < 2 * kTile) {
    const int row = tid >> 1, w = 2 * tj + (tid & 1);
    const int gi = ti * kTile + row;
    if (gi < a.n_nodes && w < n_words) a.adj[(int64_t)gi * n_words + w] = words[tid];
  }
}

__global__ void graph_degree_kernel(GraphArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_nodes) return;
  const int n_words = (a.n_nodes + 31) / 32;
  int d = 0;
  for (int w = 0; w < n_words; ++w) d += __popc(a.adj[(int64_t)i * n_words + w]);
  a.degree[i] = d;
}

__global__ void hyperplane_kernel(int n, const double* __restrict__ X, int n_obst, const double* __restrict__ lo,
                                  const double* __restrict__ hi, int32_t* idx, double* point, double* plane) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = X[3 * (int64_t)i], y = X[3 * (int64_t)i + 1], z = X[3 * (int64_t)i + 2];
  double best = __builtin_huge_val(), px = x, py = y, pz = z;
  int bi = -1;
  for (int o = 0; o < n_obst; ++o) {
    const double cx = fmin(fmax(x, lo[3 * o]), hi[3 * o]);
    const double cy = fmin(fmax(y, lo[3 * o + 1]), hi[3 * o + 1]);
    const double cz = fmin(fmax(z, lo[3 * o + 2]), hi[3 * o + 2]);
    const double d2 = (x - cx) * (x - cx) + (y - cy) * (y - cy) + (z - cz) * (z - cz);
    if (d2 < best) { best = d2; bi = o; px = cx; py = cy; pz = cz; }
  }
  idx[i] = bi;
  point[3 * (int64_t)i] = px; point[3 * (int64_t)i + 1] = py; point[3 * (int64_t)i + 2] = pz;
  const double dx = x - px, dy = y - py, dz = z - pz;
  const double nn = sqrt(dx * dx + dy * dy + dz * dz);
  double nx = 0.0, ny = 0.0, nz = 0.0;
  if (nn > 0.0) { nx = dx / nn; ny = dy / nn; nz = dz / nn; }
  plane[4 * (int64_t)i] = nx; plane[4 * (int64_t)i + 1] = ny; plane[4 * (int64_t)i + 2] = nz;
  plane[4 * (int64_t)i + 3] = nx * px + ny * py + nz * pz;
}

}  // namespace

hipError_t launch_graph(const GraphArgs& a, hipStream_t s) {
  if (a.n_nodes <= 0) return hipSuccess;
  const int64_t nm = (int64_t)a.n_nodes * a.m;
  hipLaunchKernelGGL(graph_rows_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, a);
  const int n_tiles = (a.n_nodes + kTile - 1) / kTile;
  hipLaunchKernelGGL(graph_bounds_kernel, dim3((n_tiles * a.m + 255) / 256), dim3(256), 0, s, a, n_tiles);
  hipLaunchKernelGGL(graph_pairs_kernel, dim3(n_tiles, n_tiles), dim3(256), 0, s, a);
  hipLaunchKernelGGL(graph_degree_kernel, dim3((a.n_nodes + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t graph_scratch(double** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptr[dev] = p;
  }
  *out = static_cast<double*>(ptr[dev]);
  return hipSuccess;
}

hipError_t launch_hyperplanes(int n, const double* X, int n_obst, const double* lo, const double* hi, int32_t* idx,
                              double* point, double* plane, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(hyperplane_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, X, n_obst, lo, hi, idx, point, plane);
  return hipGetLastError();
}

}  // namespace rbp
