// Comparison regularizers of Sec. V as prior agents of Alg. 2: the l_{2,1}
// agent (l2 over each range slice's cross-range plane, l1 over range) and
// the isotropic total-variation agent, each the proximal map of its
// regularizer on the prior agent's image.
//
// l_{2,1}: each range slice z is scaled by max(0, 1 - tau / ||v_z||_2): one
// pass of block partial sums of squares per slice, one pass that sums a
// slice's partials (fixed order, float64) and scales its voxels.
//
// TV: argmin_r lam TV(r) + ||r - v||^2 / 2 with TV the isotropic 3D total
// variation (forward differences, the difference leaving the volume zero),
// by `iters` steps of Chambolle's dual projection iteration from p = 0:
//   u = div p - v / lam;  g = grad u;  p <- (p + tau g) / (1 + tau |g|),
// then r = v - lam div p, with div the negative adjoint of grad and tau =
// 1/12 (the step that converges in three dimensions).  Each step is two
// voxel-per-thread stencil passes (div, then grad and the projection): a
// step reads p at a voxel's backward neighbours, which other threads of the
// same pass would be rewriting.
#include "passes.hpp"

namespace clampk {

namespace {

constexpr int kL21Chunk = 16 * kBlock;  // voxels of a slice per partial-sum block

struct Vol {
    int nx, ny, nz;
};

__device__ __forceinline__ void voxel_coords(const Vol& d, unsigned i, int& x, int& y, int& z) {
    x = (int)(i % (unsigned)d.nx);
    const unsigned q = i / (unsigned)d.nx;
    y = (int)(q % (unsigned)d.ny);
    z = (int)(q / (unsigned)d.ny);
}

// Component a of the divergence at one voxel: q[i] - q[i - 1] inside, q[0]
// at the first index, -q[n - 2] at the last, 0 along an axis of length 1.
__device__ __forceinline__ float div_axis(const float* q, unsigned i, int pos, int len, unsigned stride) {
    if (len == 1) return 0.f;
    if (pos == 0) return q[i];
    if (pos == len - 1) return -q[i - stride];
    return q[i] - q[i - stride];
}

__device__ __forceinline__ float div3_voxel(const Vol& d, const float* p, size_t n, unsigned i) {
    int x, y, z;
    voxel_coords(d, i, x, y, z);
    const unsigned sx = 1u, sy = (unsigned)d.nx, sz = (unsigned)d.nx * (unsigned)d.ny;
    return div_axis(p, i, z, d.nz, sz) + div_axis(p + n, i, y, d.ny, sy) + div_axis(p + 2 * n, i, x, d.nx, sx);
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_l21_sums(int per, int chunks, const float* in, double* part) {
    const int z = blockIdx.y, c = blockIdx.x;
    const float* v = in + (size_t)z * per;
    const int end = (c + 1) * kL21Chunk < per ? (c + 1) * kL21Chunk : per;
    float f = 0.f;
    for (int i = c * kL21Chunk + (int)threadIdx.x; i < end; i += kBlock) f += v[i] * v[i];
    double acc[1] = {f};
    block_sum_store<1>(acc, part + (size_t)z * chunks + c);
}

__global__ __launch_bounds__(kBlock) void k_l21_shrink(int per, int chunks, float tau, const double* part,
                                                       const float* in, float* out) {
    const int z = blockIdx.y, c = blockIdx.x;
    __shared__ float scale;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < chunks; ++k) s += part[(size_t)z * chunks + k];
        const double nrm = sqrt(s);
        scale = nrm > 0.0 ? (float)fmax(0.0, 1.0 - (double)tau / nrm) : 0.f;
    }
    __syncthreads();
    const float sc = scale;
    const float* v = in + (size_t)z * per;
    float* o = out + (size_t)z * per;
    const int end = (c + 1) * kL21Chunk < per ? (c + 1) * kL21Chunk : per;
    for (int i = c * kL21Chunk + (int)threadIdx.x; i < end; i += kBlock) o[i] = sc * v[i];
}

// u = div p - v / lam   (zero_p: p is zero, so u = -v / lam, and p is zeroed)
__global__ __launch_bounds__(kBlock) void k_tv_div(Vol d, size_t n, float inv_lam, int zero_p, float* p,
                                                   const float* v, float* u) {
    const unsigned i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (zero_p) {
        p[i] = 0.f;
        p[n + i] = 0.f;
        p[2 * n + i] = 0.f;
        u[i] = -v[i] * inv_lam;
    } else {
        u[i] = div3_voxel(d, p, n, i) - v[i] * inv_lam;
    }
}

// g = grad u (forward differences, 0 leaving the volume); p <- (p + tau g) / (1 + tau |g|)
__global__ __launch_bounds__(kBlock) void k_tv_step(Vol d, size_t n, float tau, const float* u, float* p) {
    const unsigned i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int x, y, z;
    voxel_coords(d, i, x, y, z);
    const float ui = u[i];
    const float gz = z < d.nz - 1 ? u[i + (unsigned)d.nx * (unsigned)d.ny] - ui : 0.f;
    const float gy = y < d.ny - 1 ? u[i + (unsigned)d.nx] - ui : 0.f;
    const float gx = x < d.nx - 1 ? u[i + 1u] - ui : 0.f;
    const float den = 1.f + tau * sqrtf(gz * gz + gy * gy + gx * gx);
    p[i] = (p[i] + tau * gz) / den;
    p[n + i] = (p[n + i] + tau * gy) / den;
    p[2 * n + i] = (p[2 * n + i] + tau * gx) / den;
}

// r = v - lam div p
__global__ __launch_bounds__(kBlock) void k_tv_out(Vol d, size_t n, float lam, const float* p, const float* v,
                                                   float* out) {
    const unsigned i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    out[i] = v[i] - lam * div3_voxel(d, p, n, i);
}

int l21_chunks(int nx, int ny) { return (nx * ny + kL21Chunk - 1) / kL21Chunk; }

hipError_t launch_prior_l21(int nx, int ny, int nz, float tau, const float* in, float* out, double* part,
                            hipStream_t st) {
    const int per = nx * ny, chunks = l21_chunks(nx, ny);
    hipLaunchKernelGGL(k_l21_sums, dim3(chunks, nz), dim3(kBlock), 0, st, per, chunks, in, part);
    hipLaunchKernelGGL(k_l21_shrink, dim3(chunks, nz), dim3(kBlock), 0, st, per, chunks, tau, part, in, out);
    return hipGetLastError();
}

hipError_t launch_prior_tv(int nx, int ny, int nz, float lam, int iters, const float* in, float* out, float* p,
                           float* u, hipStream_t st) {
    const Vol d{nx, ny, nz};
    const size_t n = (size_t)nx * ny * nz;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    const float tau = 1.f / 12.f;
    if (iters <= 0) {
        hipLaunchKernelGGL(k_tv_div, grid, dim3(kBlock), 0, st, d, n, 1.f / lam, 1, p, in, u);
    }
    for (int k = 0; k < iters; ++k) {
        hipLaunchKernelGGL(k_tv_div, grid, dim3(kBlock), 0, st, d, n, 1.f / lam, k == 0 ? 1 : 0, p, in, u);
        hipLaunchKernelGGL(k_tv_step, grid, dim3(kBlock), 0, st, d, n, tau, u, p);
    }
    hipLaunchKernelGGL(k_tv_out, grid, dim3(kBlock), 0, st, d, n, lam, p, in, out);
    return hipGetLastError();
}

}  // namespace clampk
