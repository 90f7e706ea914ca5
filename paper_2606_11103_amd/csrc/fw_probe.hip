// Memory-traffic probes: the per-cell streams of the step's updates moved
// with none of the method's arithmetic, in the two access orders a step
// kernel can use.  They measure what a schedule can reach at best: the
// velocity update's streams, the pressure update's, and the single pass a
// fused update would need, each either in one flat sweep over the grid
// (every concurrent workgroup on neighbouring cells, as the plane-major
// kernels) or by 64 x 4 tiles marching 48 planes (the pattern a fused
// update needs, since its pressure half depends on velocities of the
// following planes).  Values are written back unchanged (x + 0 * p, which
// the compiler cannot fold away), so the state is preserved.
#include "fw_internal.h"
#include "fw_vec.h"

namespace fw {

namespace {

// MODE 0: velocity streams (read p, class, v, psi1; write v, psi1)
// MODE 1: pressure streams (read v, p, class, psi2; write p, psi2)
// MODE 2: both in one pass (every state float read and written once)
// MODE 3: MODE 0 with the three per-axis psi1 groups of a cell stored together
//         ([cell][axis][N] over the psi1 arrays' memory), one stream instead of three
// MODE 4: MODE 3 with v stored [cell][axis] as well
// MODE 5: MODE 0 with the psi1 arrays blocked by 64 cells: [cell / 64][axis]
//         [cell % 64][N], so a wave's three axis groups are 3 KB in a row
//         (one stream, every load instruction on whole lines)
// MODE 6: MODE 5 with v blocked the same way ([cell / 64][axis][cell % 64])
template <int N, int MODE>
__device__ __forceinline__ void probe_cell(const Fields &F, int64_t g)
{
    // every load first (the stores may alias them), then every store
    constexpr bool ILV1 = MODE == 3 || MODE == 4, ILV_V = MODE == 4;
    constexpr bool BLK1 = MODE >= 5, BLK_V = MODE == 6;
    const int64_t blk = g >> 6, lane = g & 63;
    float *vp[3], *psi1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        vp[a] = ILV_V ? F.vx + g * 3 + a
              : BLK_V ? F.vx + (blk * 3 + a) * 64 + lane
                      : (a == 0 ? F.vx : (a == 1 ? F.vy : F.vz)) + g;
        psi1[a] = ILV1 ? F.psi1x + (g * 3 + a) * N
                : BLK1 ? F.psi1x + ((blk * 3 + a) * 64 + lane) * N
                       : (a == 0 ? F.psi1x : (a == 1 ? F.psi1y : F.psi1z)) + g * N;
    }
    const float p = load1_stream(F.p + g);
    const float c = (float)F.cls[g];
    float v[3], q1[3][N], q2[N];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = load1_stream(vp[a]);
    if constexpr (MODE != 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) load_stream<N>(psi1[a], q1[a]);
    }
    if constexpr (MODE != 0) load_stream<N>(F.psi2 + g * N, q2);
    // x + 0 * y cannot be folded away (NaN), so each store keeps its load
    if constexpr (MODE != 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int i = 0; i < N; ++i) q1[a][i] = fmaf(0.0f, p, q1[a][i]);
            store_stream<N>(psi1[a], q1[a]);
            store1_stream(vp[a], fmaf(0.0f, p + c, v[a]));
        }
    }
    if constexpr (MODE != 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) q2[i] = fmaf(0.0f, p, q2[i]);
        store_stream<N>(F.psi2 + g * N, q2);
        store1_stream(F.p + g, fmaf(0.0f, v[0] + v[1] + v[2] + c, p));
    }
}

template <int N, int MODE>
__global__ __launch_bounds__(256) void k_probe_flat(const Fields F, int64_t n)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g < n) probe_cell<N, MODE>(F, g);
}

// 64 x 4 tiles marching `chunk` planes; XCD k (block % 8) takes a contiguous
// run of the tile list, x fastest, then y, then the chunk
template <int N, int MODE>
__global__ __launch_bounds__(256) void k_probe_march(const Fields F, int nx, int px, int ny, int nz, int chunk,
                                                     int n_tiles, int per_xcd)
{
    const int b = blockIdx.x;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= n_tiles) return;
    const int ntx = (nx + 63) / 64, nty = (ny + 3) / 4;
    const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    const int x = tx * 64 + (int)threadIdx.x, y = ty * 4 + (int)threadIdx.y;
    if (x >= nx || y >= ny) return;
    const int z0 = tz * chunk, z1 = min(nz, z0 + chunk);
    for (int z = z0; z < z1; ++z) probe_cell<N, MODE>(F, ((int64_t)z * ny + y) * px + x);
}

template <int N>
hipError_t probe_n(int mode, int order, const Fields &F, int64_t nx, int64_t px, int64_t ny, int64_t nz,
                   hipStream_t s)
{
    if (order == 0) {
        const int64_t n = px * ny * nz;          // every stored cell, row padding included
        const dim3 grid((unsigned)((n + 255) / 256));
        if (mode == 0) k_probe_flat<N, 0><<<grid, dim3(256), 0, s>>>(F, n);
        if (mode == 1) k_probe_flat<N, 1><<<grid, dim3(256), 0, s>>>(F, n);
        if (mode == 2) k_probe_flat<N, 2><<<grid, dim3(256), 0, s>>>(F, n);
        if (mode == 3) k_probe_flat<N, 3><<<grid, dim3(256), 0, s>>>(F, n);
        if (mode == 4) k_probe_flat<N, 4><<<grid, dim3(256), 0, s>>>(F, n);
        if (mode == 5) k_probe_flat<N, 5><<<grid, dim3(256), 0, s>>>(F, n);
        if (mode == 6) k_probe_flat<N, 6><<<grid, dim3(256), 0, s>>>(F, n);
    } else {
        const int chunk = 48;
        const int64_t tiles = ((nx + 63) / 64) * ((ny + 3) / 4) * ((nz + chunk - 1) / chunk);
        const int per_xcd = (int)((tiles + 7) / 8);
        const dim3 grid((unsigned)(8 * per_xcd)), block(64, 4);
        if (mode == 0) k_probe_march<N, 0><<<grid, block, 0, s>>>(F, (int)nx, (int)px, (int)ny, (int)nz, chunk, (int)tiles, per_xcd);
        if (mode == 1) k_probe_march<N, 1><<<grid, block, 0, s>>>(F, (int)nx, (int)px, (int)ny, (int)nz, chunk, (int)tiles, per_xcd);
        if (mode == 2) k_probe_march<N, 2><<<grid, block, 0, s>>>(F, (int)nx, (int)px, (int)ny, (int)nz, chunk, (int)tiles, per_xcd);
        if (mode == 3) k_probe_march<N, 3><<<grid, block, 0, s>>>(F, (int)nx, (int)px, (int)ny, (int)nz, chunk, (int)tiles, per_xcd);
        if (mode == 4) k_probe_march<N, 4><<<grid, block, 0, s>>>(F, (int)nx, (int)px, (int)ny, (int)nz, chunk, (int)tiles, per_xcd);
        if (mode == 5) k_probe_march<N, 5><<<grid, block, 0, s>>>(F, (int)nx, (int)px, (int)ny, (int)nz, chunk, (int)tiles, per_xcd);
        if (mode == 6) k_probe_march<N, 6><<<grid, block, 0, s>>>(F, (int)nx, (int)px, (int)ny, (int)nz, chunk, (int)tiles, per_xcd);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stream_probe(int nmech, int mode, int order, const Fields &F, int64_t nx, int64_t px, int64_t ny,
                               int64_t nz, hipStream_t s)
{
    if (mode < 0 || mode > 6 || order < 0 || order > 1) return hipErrorInvalidValue;
    switch (nmech) {
    case 1: return probe_n<1>(mode, order, F, nx, px, ny, nz, s);
    case 2: return probe_n<2>(mode, order, F, nx, px, ny, nz, s);
    case 3: return probe_n<3>(mode, order, F, nx, px, ny, nz, s);
    case 4: return probe_n<4>(mode, order, F, nx, px, ny, nz, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fw
