// Initial state, diagnostics reductions and the streaming copy kernel.
#include "gs_device.hpp"
#include "gs_launch.hpp"

namespace gs {

// ------------------------------------------------------------------ init
// u = 1, v = 0 everywhere except the axis-aligned cube [c0, c0 + side) per
// axis with c0 = floor((n - side) / 2), which holds (cu, cv). Values are
// rounded to FP32 first and then to the 16-bit storage types.
template <typename S>
__global__ __launch_bounds__(256) void init_cube_kernel(S *__restrict__ u, S *__restrict__ v, int nx, int ny,
                                                        int nz, int side, double cu, double cv)
{
    const size_t n = (size_t)nx * ny * nz;
    const int x0 = (nx - side) / 2, y0 = (ny - side) / 2, z0 = (nz - side) / 2;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const size_t r = i / nx;
        const int y = (int)(r % ny);
        const int z = (int)(r / ny);
        const bool in = x >= x0 && x < x0 + side && y >= y0 && y < y0 + side && z >= z0 && z < z0 + side;
        typedef typename Traits<S>::C C;
        const C a = in ? (C)cu : (C)1;
        const C b = in ? (C)cv : (C)0;
        u[i] = fstore<S>(0, a);
        v[i] = fstore<S>(1, b);
    }
}

static unsigned grid_for(size_t n, unsigned per_block, unsigned cap)
{
    size_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

hipError_t launch_init_cube(int storage, void *u, void *v, int nx, int ny, int nz, int side, double cu,
                            double cv, hipStream_t st)
{
    const size_t n = (size_t)nx * ny * nz;
    const unsigned g = grid_for(n, 256, 65536);
    switch (storage) {
    case 0: hipLaunchKernelGGL(init_cube_kernel<double>, dim3(g), dim3(256), 0, st, (double *)u, (double *)v, nx, ny, nz, side, cu, cv); break;
    case 1: hipLaunchKernelGGL(init_cube_kernel<float>, dim3(g), dim3(256), 0, st, (float *)u, (float *)v, nx, ny, nz, side, cu, cv); break;
    case 2: hipLaunchKernelGGL(init_cube_kernel<bf16>, dim3(g), dim3(256), 0, st, (bf16 *)u, (bf16 *)v, nx, ny, nz, side, cu, cv); break;
    case 4: hipLaunchKernelGGL(init_cube_kernel<bf16c>, dim3(g), dim3(256), 0, st, (bf16c *)u, (bf16c *)v, nx, ny, nz, side, cu, cv); break;
    case 3: hipLaunchKernelGGL(init_cube_kernel<f16>, dim3(g), dim3(256), 0, st, (f16 *)u, (f16 *)v, nx, ny, nz, side, cu, cv); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Periodic box [x0, x0 + side) x [y0, y0 + side) x [z0, z0 + side) (wrapping
// around the grid) holds (cu, cv); every other cell (1, 0).
template <typename S>
__global__ __launch_bounds__(256) void init_box_kernel(S *__restrict__ u, S *__restrict__ v, int nx, int ny, int nz,
                                                       int x0, int y0, int z0, int side, double cu, double cv)
{
    const size_t n = (size_t)nx * ny * nz;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const size_t r = i / nx;
        const int y = (int)(r % ny);
        const int z = (int)(r / ny);
        const int dx = (x - x0 + nx) % nx, dy = (y - y0 + ny) % ny, dz = (z - z0 + nz) % nz;
        const bool in = dx < side && dy < side && dz < side;
        typedef typename Traits<S>::C C;
        u[i] = fstore<S>(0, in ? (C)cu : (C)1);
        v[i] = fstore<S>(1, in ? (C)cv : (C)0);
    }
}

hipError_t launch_init_box(int storage, void *u, void *v, int nx, int ny, int nz, int x0, int y0, int z0, int side,
                           double cu, double cv, hipStream_t st)
{
    const size_t n = (size_t)nx * ny * nz;
    const unsigned g = grid_for(n, 256, 65536);
    switch (storage) {
    case 0: hipLaunchKernelGGL(init_box_kernel<double>, dim3(g), dim3(256), 0, st, (double *)u, (double *)v, nx, ny, nz, x0, y0, z0, side, cu, cv); break;
    case 1: hipLaunchKernelGGL(init_box_kernel<float>, dim3(g), dim3(256), 0, st, (float *)u, (float *)v, nx, ny, nz, x0, y0, z0, side, cu, cv); break;
    case 2: hipLaunchKernelGGL(init_box_kernel<bf16>, dim3(g), dim3(256), 0, st, (bf16 *)u, (bf16 *)v, nx, ny, nz, x0, y0, z0, side, cu, cv); break;
    case 4: hipLaunchKernelGGL(init_box_kernel<bf16c>, dim3(g), dim3(256), 0, st, (bf16c *)u, (bf16c *)v, nx, ny, nz, x0, y0, z0, side, cu, cv); break;
    case 3: hipLaunchKernelGGL(init_box_kernel<f16>, dim3(g), dim3(256), 0, st, (f16 *)u, (f16 *)v, nx, ny, nz, x0, y0, z0, side, cu, cv); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Sum over i of (a_i - b_i)^2 in FP64: per-workgroup partials (fixed tree).
template <typename S>
__global__ __launch_bounds__(256) void sqdiff_partial(const S *__restrict__ a, const S *__restrict__ b, size_t n,
                                                      double *__restrict__ part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double d = (double)Traits<S>::load(a[i]) - (double)Traits<S>::load(b[i]);
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

int sqdiff_blocks() { return 512; }

hipError_t launch_sqdiff(int storage, const void *a, const void *b, size_t n, double *part, hipStream_t st)
{
    const unsigned g = sqdiff_blocks();
    switch (storage) {
    case 0: hipLaunchKernelGGL(sqdiff_partial<double>, dim3(g), dim3(256), 0, st, (const double *)a, (const double *)b, n, part); break;
    case 1: hipLaunchKernelGGL(sqdiff_partial<float>, dim3(g), dim3(256), 0, st, (const float *)a, (const float *)b, n, part); break;
    case 2:
    case 4: // (1 - a) - (1 - b) = b - a exactly: the complemented u needs no conversion here
        hipLaunchKernelGGL(sqdiff_partial<bf16>, dim3(g), dim3(256), 0, st, (const bf16 *)a, (const bf16 *)b, n, part); break;
    case 3: hipLaunchKernelGGL(sqdiff_partial<f16>, dim3(g), dim3(256), 0, st, (const f16 *)a, (const f16 *)b, n, part); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ diagnostics
// Neumaier-compensated FP64 accumulation; every reduction tree below has a
// fixed shape, so results do not depend on scheduling.
struct Acc {
    double su, cu, sv, cv;
    double mnu, mxu, mnv, mxv;
    double nonfinite;
};

__device__ __forceinline__ void neumaier_add(double &s, double &c, double x)
{
    const double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

__device__ __forceinline__ void acc_merge(Acc &a, const Acc &b)
{
    neumaier_add(a.su, a.cu, b.su);
    a.cu += b.cu;
    neumaier_add(a.sv, a.cv, b.sv);
    a.cv += b.cv;
    a.mnu = fmin(a.mnu, b.mnu);
    a.mxu = fmax(a.mxu, b.mxu);
    a.mnv = fmin(a.mnv, b.mnv);
    a.mxv = fmax(a.mxv, b.mxv);
    a.nonfinite += b.nonfinite;
}

__device__ __forceinline__ Acc acc_empty()
{
    Acc a;
    a.su = a.cu = a.sv = a.cv = 0.0;
    a.mnu = a.mnv = __builtin_inf();
    a.mxu = a.mxv = -__builtin_inf();
    a.nonfinite = 0.0;
    return a;
}

__device__ __forceinline__ Acc acc_shfl_xor(const Acc &a, int lane_mask)
{
    Acc b;
    b.su = __shfl_xor(a.su, lane_mask, 64);
    b.cu = __shfl_xor(a.cu, lane_mask, 64);
    b.sv = __shfl_xor(a.sv, lane_mask, 64);
    b.cv = __shfl_xor(a.cv, lane_mask, 64);
    b.mnu = __shfl_xor(a.mnu, lane_mask, 64);
    b.mxu = __shfl_xor(a.mxu, lane_mask, 64);
    b.mnv = __shfl_xor(a.mnv, lane_mask, 64);
    b.mxv = __shfl_xor(a.mxv, lane_mask, 64);
    b.nonfinite = __shfl_xor(a.nonfinite, lane_mask, 64);
    return b;
}

// Butterfly within the 64-lane wavefront, then the 4 wavefronts in order.
// Every lane of wave 0 ends with the same block total; lane 0 returns it.
__device__ Acc block_reduce(Acc a)
{
    __shared__ Acc part[4];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        Acc o = acc_shfl_xor(a, m);
        // combine in lane order (lower lane's value first) for symmetry
        const bool low = (threadIdx.x & m) == 0;
        Acc x = low ? a : o, y = low ? o : a;
        acc_merge(x, y);
        a = x;
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) part[w] = a;
    __syncthreads();
    Acc r = part[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) acc_merge(r, part[i]);
    return r;
}

// Stored value of field f (0 = u, 1 = v) as FP64 (for the complemented storage
// 1 - stored u, exact in FP64).
template <typename S>
__device__ __forceinline__ double as_f64(int f, S x)
{
    const double d = (double)Traits<S>::load(x);
    if constexpr (Complemented<S>::value) return f == 0 ? 1.0 - d : d;
    else return d;
}

static constexpr int k_diag_blocks = 1024;
static constexpr int k_diag_fields = 9;

template <typename S>
__global__ __launch_bounds__(256) void diag_partial(const S *__restrict__ u, const S *__restrict__ v, size_t n,
                                                    double *__restrict__ part)
{
    Acc a = acc_empty();
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double x = as_f64(0, u[i]), y = as_f64(1, v[i]);
        if (isfinite(x)) {
            neumaier_add(a.su, a.cu, x);
            a.mnu = fmin(a.mnu, x);
            a.mxu = fmax(a.mxu, x);
        } else {
            a.nonfinite += 1.0;
        }
        if (isfinite(y)) {
            neumaier_add(a.sv, a.cv, y);
            a.mnv = fmin(a.mnv, y);
            a.mxv = fmax(a.mxv, y);
        } else {
            a.nonfinite += 1.0;
        }
    }
    const Acc r = block_reduce(a);
    if (threadIdx.x == 0) {
        double *o = part + (size_t)blockIdx.x * k_diag_fields;
        o[0] = r.su; o[1] = r.cu; o[2] = r.sv; o[3] = r.cv;
        o[4] = r.mnu; o[5] = r.mxu; o[6] = r.mnv; o[7] = r.mxv; o[8] = r.nonfinite;
    }
}

__global__ __launch_bounds__(256) void diag_final(const double *__restrict__ part, int nparts, double *__restrict__ out)
{
    Acc a = acc_empty();
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        const double *p = part + (size_t)i * k_diag_fields;
        Acc b;
        b.su = p[0]; b.cu = p[1]; b.sv = p[2]; b.cv = p[3];
        b.mnu = p[4]; b.mxu = p[5]; b.mnv = p[6]; b.mxv = p[7]; b.nonfinite = p[8];
        acc_merge(a, b);
    }
    const Acc r = block_reduce(a);
    if (threadIdx.x == 0) {
        out[0] = r.su; out[1] = r.cu; out[2] = r.sv; out[3] = r.cv;
        out[4] = r.mnu; out[5] = r.mxu; out[6] = r.mnv; out[7] = r.mxv; out[8] = r.nonfinite;
    }
}

size_t diag_workspace_bytes() { return (size_t)(k_diag_blocks + 1) * k_diag_fields * sizeof(double); }
size_t diag_result_offset() { return (size_t)k_diag_blocks * k_diag_fields * sizeof(double); }

hipError_t launch_diagnostics(int storage, const void *u, const void *v, size_t n, void *ws, hipStream_t st)
{
    double *part = (double *)ws;
    double *out = (double *)((char *)ws + diag_result_offset());
    const unsigned g = k_diag_blocks;
    switch (storage) {
    case 0: hipLaunchKernelGGL(diag_partial<double>, dim3(g), dim3(256), 0, st, (const double *)u, (const double *)v, n, part); break;
    case 1: hipLaunchKernelGGL(diag_partial<float>, dim3(g), dim3(256), 0, st, (const float *)u, (const float *)v, n, part); break;
    case 2: hipLaunchKernelGGL(diag_partial<bf16>, dim3(g), dim3(256), 0, st, (const bf16 *)u, (const bf16 *)v, n, part); break;
    case 4: hipLaunchKernelGGL(diag_partial<bf16c>, dim3(g), dim3(256), 0, st, (const bf16c *)u, (const bf16c *)v, n, part); break;
    case 3: hipLaunchKernelGGL(diag_partial<f16>, dim3(g), dim3(256), 0, st, (const f16 *)u, (const f16 *)v, n, part); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_final, dim3(1), dim3(256), 0, st, (const double *)part, (int)g, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ copy
// 16-byte vector copy, four independent accesses in flight per lane per trip.
__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n16)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st)
{
    const size_t n16 = bytes / 16;
    const unsigned g = grid_for(n16, 256 * 4, 256 * 64);
    hipLaunchKernelGGL(copy_kernel, dim3(g), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst, n16);
    return hipGetLastError();
}

// ------------------------------------------------------------------ counter
__global__ void set_u64_kernel(uint64_t *dst, uint64_t value)
{
    if (threadIdx.x == 0) *dst = value;
}

hipError_t launch_set_u64(uint64_t *dst, uint64_t value, hipStream_t st)
{
    hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, st, dst, value);
    return hipGetLastError();
}

} // namespace gs
