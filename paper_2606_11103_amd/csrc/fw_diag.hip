// Diagnostics of one step: the staggered-time discrete energy
//   E^{n+1/2} = 1/2 sum_faces rho_f |v^{n+1/2}|^2 + 1/2 sum_cells p^{n+1} p^n / K,
// which the lossless scheme conserves exactly (div = -grad^T), the largest
// |p^{n+1}| and the number of non-finite pressures.  FP64 accumulation per
// thread and per block in a fixed order; one partial per tile, summed per
// domain on the host.
#include <algorithm>

#include "fw_internal.h"
#include "fw_vec.h"

namespace fw {

namespace {

template <int NDIM>
__global__ __launch_bounds__(1024) void k_energy(const StepArgs A, const float *__restrict__ p_old, double *partial)
{
    __shared__ double s_e[1024];
    __shared__ float s_m[1024];
    __shared__ int s_nf[1024];
    const int b = blockIdx.x;
    const int ti = (b & 7) * A.tiles_per_xcd + (b >> 3);
    if (ti >= A.n_tiles) return;
    const Tile T = A.tiles[ti];
    const DomainDesc D = A.doms[T.dom];
    const int nx = (int)D.n[0], ny = (int)D.n[1], nz = (int)D.n[2], px = D.pitch;
    const int st[3] = {1, px, px * ny};
    const int nn[3] = {nx, ny, nz};
    const int64_t o = D.cell_off;
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int x = T.x0 + (int)threadIdx.x;
    int y = NDIM == 3 ? T.y0 + (int)threadIdx.y : 0;
    double e = 0.0;
    float mx = 0.0f;
    int nf = 0;
    const float *vv[3] = {A.f.vx + o, A.f.vy + o, A.f.vz + o};
    if (x < nx && y < ny) {
        for (int z = T.z0; z < T.z1; ++z) {
            int c[3] = {x, y, 0};
            if (NDIM == 3) c[2] = z;
            if (NDIM == 2) c[1] = z;
            const int g = (c[2] * ny + c[1]) * px + c[0];        // stored index
            const int u = (c[2] * ny + c[1]) * nx + c[0];        // unpadded index (speed perturbation)
            const int L = A.f.cls[o + g];
            const ClassCoef &cc = A.classes[D.class_base + L];
            float K = cc.K;
            if (A.noise_amp != 0.0f) K = K * speed_factor_sq(D.noise_seed, (uint32_t)u, A.noise_amp);
            const float pn = A.f.p[o + g];
            if (!isfinite(pn)) ++nf;
            mx = fmaxf(mx, fabsf(pn));
            e += 0.5 * (double)pn * (double)p_old[o + g] / (double)K;
#pragma unroll
            for (int a = 0; a < NDIM; ++a) {
                const int Ln = (c[a] + 1 < nn[a]) ? A.f.cls[o + g + st[a]] : L;
                const double rf = 0.5 * ((double)cc.rho + (double)A.classes[D.class_base + Ln].rho);
                const double va = vv[a][g];
                e += 0.5 * rf * va * va;
            }
        }
    }
    s_e[tid] = e;
    s_m[tid] = mx;
    s_nf[tid] = nf;
    __syncthreads();
    const int nt = blockDim.x * blockDim.y;
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w && tid + w < nt) {
            s_e[tid] += s_e[tid + w];
            s_m[tid] = fmaxf(s_m[tid], s_m[tid + w]);
            s_nf[tid] += s_nf[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        partial[3 * (int64_t)ti] = s_e[0];
        partial[3 * (int64_t)ti + 1] = (double)s_m[0];
        partial[3 * (int64_t)ti + 2] = (double)s_nf[0];
    }
}

// Streaming device-to-device copy: one 16-byte non-temporal load and store
// per lane and a grid as large as the copy (measured on MI355X: 6.6 TB/s of
// read + write traffic, against 5.3 TB/s for a grid-stride loop over 1024
// workgroups).  A dispatch covers fewer than 2^32 work-items along x, and
// the count wraps silently beyond that, so a launch moves at most 2^22
// workgroups of 256 lanes (16 GiB); larger copies take several launches.
typedef float copy_v4 __attribute__((ext_vector_type(4)));
constexpr int64_t kCopyMaxBlocks = int64_t(1) << 22;

__global__ __launch_bounds__(256) void k_copy16(const copy_v4 *__restrict__ src, copy_v4 *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Validation of a caller's map: one grid-stride pass, one atomic per block.
__global__ __launch_bounds__(256) void k_count_outside_unit(const float *__restrict__ x, int64_t n,
                                                            unsigned long long *count)
{
    __shared__ unsigned int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    unsigned int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float v = x[i];
        if (!(v >= 0.0f && v <= 1.0f)) ++bad;      // NaN fails both comparisons
    }
    if (bad) atomicAdd(&s_bad, bad);
    __syncthreads();
    if (threadIdx.x == 0 && s_bad) atomicAdd(count, (unsigned long long)s_bad);
}

}  // namespace

hipError_t launch_count_outside_unit(const float *x, int64_t n, unsigned long long *count, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(8192, (n + 255) / 256);
    k_count_outside_unit<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(x, n, count);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, int64_t bytes, hipStream_t s)
{
    if (bytes <= 0) return hipSuccess;
    const bool aligned = ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) == 0 &&
                         (bytes & 15) == 0;
    if (!aligned) return hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, s);
    const copy_v4 *in = static_cast<const copy_v4 *>(src);
    copy_v4 *out = static_cast<copy_v4 *>(dst);
    for (int64_t left = bytes / 16; left > 0;) {
        const int64_t blocks = std::min<int64_t>(kCopyMaxBlocks, (left + 255) / 256);
        const int64_t n = std::min<int64_t>(left, blocks * 256);
        k_copy16<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(in, out, n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        in += n;
        out += n;
        left -= n;
    }
    return hipSuccess;
}

hipError_t launch_energy(int ndim, const StepArgs &a, const float *p_old, double *partial, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    int tx, ty;
    tile_shape(ndim, 16, &tx, &ty);
    (void)ty;
    const dim3 grid(8 * a.tiles_per_xcd);
    if (ndim == 1) k_energy<1><<<grid, dim3(tx, 1), 0, s>>>(a, p_old, partial);
    if (ndim == 2) k_energy<2><<<grid, dim3(tx, 1), 0, s>>>(a, p_old, partial);
    if (ndim == 3) k_energy<3><<<grid, dim3(tx, a.tile_rows), 0, s>>>(a, p_old, partial);
    return hipGetLastError();
}

}  // namespace fw
