// gfx950 kernels of the FDTD step: velocity update, pressure update and the
// source/receiver step.  Paper: Sec. 2.1 (stretched pressure-velocity system,
// memory-variable recursion of Eq. relaxation_psi), Sec. 3.3 (staggered
// stencil of order 8 in space, M = 4).
//
// Work decomposition.  A tile is a 64-cell run along x (times a band of rows
// along y in 3D) that marches along the slowest axis (z in 3D, y in 2D).
// Each thread owns one column per row of the band and keeps the pressure
// (velocity-kernel) or the marching-axis velocity (pressure-kernel) of eight
// consecutive planes in registers, so the marching-axis stencil costs no
// extra memory traffic.  The x and y stencils read the current plane from LDS.
// Every output cell is written by exactly one thread with a fixed operation
// order, so results do not depend on the tiling, the batching or the launch
// path.  Blocks are mapped to tiles so that each of the eight XCDs receives a
// contiguous range of the tile list (workgroups are dispatched round-robin
// over the XCDs), keeping neighbouring tiles and their halos in one L2.
#include "fw_internal.h"

namespace fw {

namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int N>
__device__ __forceinline__ void load_vec(const float *__restrict__ src, float (&v)[N])
{
    if constexpr (N == 4) {
        const float4 t = *reinterpret_cast<const float4 *>(src);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (N == 2) {
        const float2 t = *reinterpret_cast<const float2 *>(src);
        v[0] = t.x; v[1] = t.y;
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = src[i];
    }
}

template <int N>
__device__ __forceinline__ void store_vec(float *__restrict__ dst, const float (&v)[N])
{
    if constexpr (N == 4) {
        *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (N == 2) {
        *reinterpret_cast<float2 *>(dst) = make_float2(v[0], v[1]);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) dst[i] = v[i];
    }
}

__device__ __forceinline__ int tile_index(const StepArgs &A)
{
    const int b = blockIdx.x;
    return (b & 7) * A.tiles_per_xcd + (b >> 3);
}

// One face of the velocity update along one axis: memory variables of the
// gradient operator, the CPML variable inside the slab, then v.
template <int N>
__device__ __forceinline__ void velocity_face(const StepArgs &A, int axis, float D, int L, int L1,
                                              const float *s_ik, const float *s_rho,
                                              const float (*s_a)[kMaxLocalClasses],
                                              const float (*s_b)[kMaxLocalClasses],
                                              float *__restrict__ v, float *__restrict__ psi, int64_t g,
                                              int64_t c, int64_t n, int32_t pml_off)
{
    const float m = 2.0f * A.dt / (s_rho[L] + s_rho[L1]);
    float s = s_ik[L] * D;
    float ps[N];
    load_vec<N>(psi + g * N, ps);
#pragma unroll
    for (int nu = 0; nu < N; ++nu) {
        ps[nu] = s_b[nu][L] * ps[nu] + s_a[nu][L] * D;
        s += ps[nu];
    }
    store_vec<N>(psi + g * N, ps);
    if (A.pml > 0 && (c < A.pml || c >= n - A.pml)) {
        const float aF = A.pml_tab[pml_off + c];
        const float bF = A.pml_tab[pml_off + n + c];
        float *pp = A.f.pP1[axis];
        const float q = bF * pp[g] + aF * D;
        pp[g] = q;
        s += q;
    }
    v[g] -= m * s;
}

template <int NDIM, int N, int BX, int BY, int RY>
__global__ __launch_bounds__(BX *BY) void k_velocity(const StepArgs A)
{
    constexpr int TY = NDIM == 3 ? BY * RY : 1;
    constexpr int LX = BX + 8;
    constexpr int LY = NDIM == 3 ? TY + 8 : 1;
    constexpr int NT = BX * BY;
    constexpr int CX = BX + 1;
    constexpr int NHALO = NDIM == 3 ? 8 * LX + 8 * TY : 8;
    constexpr int NCHALO = NDIM == 3 ? TY + BX : 1;
    static_assert(NDIM == 3 || (BY == 1 && RY == 1), "bands of rows are 3D only");
    __shared__ float sp[LY * LX];
    __shared__ uint8_t scl[(TY + 1) * CX];
    __shared__ float s_ik[kMaxLocalClasses], s_rho[kMaxLocalClasses];
    __shared__ float s_a[N][kMaxLocalClasses], s_b[N][kMaxLocalClasses];

    const int ti = tile_index(A);
    if (ti >= A.n_tiles) return;
    const Tile T = A.tiles[ti];
    const DomainDesc D = A.doms[T.dom];
    const int tid = threadIdx.y * BX + threadIdx.x;
    for (int c = tid; c < D.n_classes; c += NT) {
        const ClassCoef &cc = A.classes[D.class_base + c];
        s_ik[c] = cc.ik1;
        s_rho[c] = cc.rho;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            s_a[nu][c] = cc.a1[nu];
            s_b[nu][c] = cc.b1[nu];
        }
    }

    const int64_t nx = D.n[0], ny = D.n[1];
    const int64_t nmarch = NDIM == 3 ? D.n[2] : (NDIM == 2 ? D.n[1] : 1);
    const int64_t sm = NDIM == 3 ? nx * ny : nx;
    const int64_t base = D.cell_off;
    const float *__restrict__ p = A.f.p;
    const uint8_t *__restrict__ cls = A.f.cls;
    float *__restrict__ vmarch = NDIM == 3 ? A.f.vz : A.f.vy;
    float *__restrict__ psimarch = NDIM == 3 ? A.f.psi1z : A.f.psi1y;
    const int tx = threadIdx.x;
    const int64_t x = T.x0 + tx;

    int64_t yr[RY], col[RY];
    bool ok[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        yr[r] = NDIM == 3 ? T.y0 + threadIdx.y * RY + r : 0;
        ok[r] = x < nx && (NDIM < 3 || yr[r] < ny);
        col[r] = base + (NDIM == 3 ? yr[r] * nx : 0) + x;
    }

    float q[RY][8];
    int cq[RY][2];
    const int z0 = T.z0;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
#pragma unroll
        for (int j = 0; j < 8; ++j) q[r][j] = 0.0f;
        cq[r][0] = 0;
        cq[r][1] = 0;
        if constexpr (NDIM >= 2) {
#pragma unroll
            for (int j = 0; j < 7; ++j) {
                const int64_t zz = z0 - 3 + j;
                q[r][j] = (ok[r] && zz >= 0 && zz < nmarch) ? p[col[r] + zz * sm] : 0.0f;
            }
            cq[r][0] = ok[r] ? cls[col[r] + z0 * sm] : 0;
        }
    }

    for (int z = z0; z < T.z1; ++z) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if constexpr (NDIM >= 2) {
                const int64_t zz = z + 4;
                q[r][7] = (ok[r] && zz < nmarch) ? p[col[r] + zz * sm] : 0.0f;
                cq[r][1] = (ok[r] && z + 1 < nmarch) ? cls[col[r] + (z + 1) * sm] : cq[r][0];
            } else {
                q[r][3] = ok[r] ? p[col[r]] : 0.0f;
                cq[r][0] = ok[r] ? cls[col[r]] : 0;
            }
            const int row = NDIM == 3 ? threadIdx.y * RY + r : 0;
            sp[(NDIM == 3 ? row + 4 : 0) * LX + 4 + tx] = q[r][3];
            scl[row * CX + tx] = (uint8_t)cq[r][0];
        }
        const int64_t zoff = base + (int64_t)z * sm;
        for (int h = tid; h < NHALO; h += NT) {
            int hy, hx;
            if constexpr (NDIM == 3) {
                if (h < 8 * LX) {
                    const int rr = h / LX;
                    hy = rr < 4 ? rr : TY + rr;
                    hx = h - rr * LX;
                } else {
                    const int hh = h - 8 * LX;
                    hy = 4 + (hh >> 3);
                    const int k = hh & 7;
                    hx = k < 4 ? k : BX + k;
                }
            } else {
                hy = 0;
                hx = h < 4 ? h : BX + h;
            }
            const int64_t gx = T.x0 - 4 + hx;
            const int64_t gy = NDIM == 3 ? T.y0 - 4 + hy : 0;
            float val = 0.0f;
            if (gx >= 0 && gx < nx && gy >= 0 && (NDIM < 3 || gy < ny))
                val = p[zoff + (NDIM == 3 ? gy * nx : 0) + gx];
            sp[hy * LX + hx] = val;
        }
        for (int h = tid; h < NCHALO; h += NT) {
            int64_t gx, gy;
            int li;
            if (h < TY) {               // column right of the band
                gx = T.x0 + BX;
                gy = NDIM == 3 ? T.y0 + h : 0;
                li = h * CX + BX;
            } else {                    // row above the band (3D)
                gx = T.x0 + (h - TY);
                gy = T.y0 + TY;
                li = TY * CX + (h - TY);
            }
            uint8_t val = 0;
            if (gx < nx && (NDIM < 3 || gy < ny)) val = cls[zoff + (NDIM == 3 ? gy * nx : 0) + gx];
            scl[li] = val;
        }
        __syncthreads();

#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!ok[r]) continue;
            const int row = NDIM == 3 ? threadIdx.y * RY + r : 0;
            const int ly = NDIM == 3 ? row + 4 : 0;
            const float *sr = sp + ly * LX + 4 + tx;
            const int64_t g = col[r] + (int64_t)z * sm;
            const int L = cq[r][0];
            {
                const float Dx = A.fd[0] * (sr[1] - sr[0]) + A.fd[1] * (sr[2] - sr[-1]) +
                                 A.fd[2] * (sr[3] - sr[-2]) + A.fd[3] * (sr[4] - sr[-3]);
                const int L1 = (x + 1 < nx) ? scl[row * CX + tx + 1] : L;
                velocity_face<N>(A, 0, Dx, L, L1, s_ik, s_rho, s_a, s_b, A.f.vx, A.f.psi1x, g, x, nx,
                                 D.pml_off[0]);
            }
            if constexpr (NDIM == 3) {
                const float Dy = A.fd[0] * (sr[LX] - sr[0]) + A.fd[1] * (sr[2 * LX] - sr[-LX]) +
                                 A.fd[2] * (sr[3 * LX] - sr[-2 * LX]) + A.fd[3] * (sr[4 * LX] - sr[-3 * LX]);
                const int L1 = (yr[r] + 1 < ny) ? scl[(row + 1) * CX + tx] : L;
                velocity_face<N>(A, 1, Dy, L, L1, s_ik, s_rho, s_a, s_b, A.f.vy, A.f.psi1y, g, yr[r], ny,
                                 D.pml_off[1]);
            }
            if constexpr (NDIM >= 2) {
                const float Dz = A.fd[0] * (q[r][4] - q[r][3]) + A.fd[1] * (q[r][5] - q[r][2]) +
                                 A.fd[2] * (q[r][6] - q[r][1]) + A.fd[3] * (q[r][7] - q[r][0]);
                const int L1 = (z + 1 < nmarch) ? cq[r][1] : L;
                velocity_face<N>(A, NDIM - 1, Dz, L, L1, s_ik, s_rho, s_a, s_b, vmarch, psimarch, g, z, nmarch,
                                 D.pml_off[NDIM - 1]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RY; ++r) {
#pragma unroll
            for (int j = 0; j < 7; ++j) q[r][j] = q[r][j + 1];
            cq[r][0] = cq[r][1];
        }
    }
}

template <int NDIM, int N, int BX, int BY, int RY>
__global__ __launch_bounds__(BX *BY) void k_pressure(const StepArgs A)
{
    constexpr int TY = NDIM == 3 ? BY * RY : 1;
    constexpr int LX = BX + 8;
    constexpr int LY = NDIM == 3 ? TY + 8 : 1;
    constexpr int NT = BX * BY;
    static_assert(NDIM == 3 || (BY == 1 && RY == 1), "bands of rows are 3D only");
    __shared__ float svx[TY * LX];
    __shared__ float svy[NDIM == 3 ? LY * BX : 1];
    __shared__ float s_ik[kMaxLocalClasses], s_K[kMaxLocalClasses], s_tb[kMaxLocalClasses];
    __shared__ float s_a[N][kMaxLocalClasses], s_b[N][kMaxLocalClasses];

    const int ti = tile_index(A);
    if (ti >= A.n_tiles) return;
    const Tile T = A.tiles[ti];
    const DomainDesc D = A.doms[T.dom];
    const int tid = threadIdx.y * BX + threadIdx.x;
    for (int c = tid; c < D.n_classes; c += NT) {
        const ClassCoef &cc = A.classes[D.class_base + c];
        s_ik[c] = cc.ik2;
        s_K[c] = cc.K;
        s_tb[c] = cc.twobeta;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            s_a[nu][c] = cc.a2[nu];
            s_b[nu][c] = cc.b2[nu];
        }
    }

    const int64_t nx = D.n[0], ny = D.n[1];
    const int64_t nmarch = NDIM == 3 ? D.n[2] : (NDIM == 2 ? D.n[1] : 1);
    const int64_t sm = NDIM == 3 ? nx * ny : nx;
    const int64_t base = D.cell_off;
    const float *__restrict__ vx = A.f.vx;
    const float *__restrict__ vy = A.f.vy;
    const float *__restrict__ vmarch = NDIM == 3 ? A.f.vz : A.f.vy;
    float *__restrict__ p = A.f.p;
    const int tx = threadIdx.x;
    const int64_t x = T.x0 + tx;

    int64_t yr[RY], col[RY];
    bool ok[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        yr[r] = NDIM == 3 ? T.y0 + threadIdx.y * RY + r : 0;
        ok[r] = x < nx && (NDIM < 3 || yr[r] < ny);
        col[r] = base + (NDIM == 3 ? yr[r] * nx : 0) + x;
    }
    float vq[RY][8];
    const int z0 = T.z0;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
#pragma unroll
        for (int j = 0; j < 8; ++j) vq[r][j] = 0.0f;
        if constexpr (NDIM >= 2) {
#pragma unroll
            for (int j = 0; j < 7; ++j) {
                const int64_t zz = z0 - 4 + j;
                vq[r][j] = (ok[r] && zz >= 0 && zz < nmarch) ? vmarch[col[r] + zz * sm] : 0.0f;
            }
        }
    }

    for (int z = z0; z < T.z1; ++z) {
        if constexpr (NDIM >= 2) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const int64_t zz = z + 3;
                vq[r][7] = (ok[r] && zz < nmarch) ? vmarch[col[r] + zz * sm] : 0.0f;
            }
        }
        const int64_t zoff = base + (int64_t)z * sm;
        for (int h = tid; h < TY * LX; h += NT) {
            const int row = h / LX;
            const int hx = h - row * LX;
            const int64_t gx = T.x0 - 4 + hx;
            const int64_t gy = NDIM == 3 ? T.y0 + row : 0;
            float val = 0.0f;
            if (gx >= 0 && gx < nx && (NDIM < 3 || gy < ny)) val = vx[zoff + (NDIM == 3 ? gy * nx : 0) + gx];
            svx[h] = val;
        }
        if constexpr (NDIM == 3) {
            for (int h = tid; h < LY * BX; h += NT) {
                const int row = h / BX;
                const int hx = h - row * BX;
                const int64_t gx = T.x0 + hx;
                const int64_t gy = T.y0 - 4 + row;
                float val = 0.0f;
                if (gx < nx && gy >= 0 && gy < ny) val = vy[zoff + gy * nx + gx];
                svy[h] = val;
            }
        }
        __syncthreads();

#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!ok[r]) continue;
            const int row = NDIM == 3 ? threadIdx.y * RY + r : 0;
            const int64_t g = col[r] + (int64_t)z * sm;
            const float *sx = svx + row * LX + 4 + tx;
            const float Dx = A.fd[0] * (sx[0] - sx[-1]) + A.fd[1] * (sx[1] - sx[-2]) +
                             A.fd[2] * (sx[2] - sx[-3]) + A.fd[3] * (sx[3] - sx[-4]);
            float Dy = 0.0f, Dz = 0.0f;
            if constexpr (NDIM == 3) {
                const float *sy = svy + (row + 4) * BX + tx;
                Dy = A.fd[0] * (sy[0] - sy[-BX]) + A.fd[1] * (sy[BX] - sy[-2 * BX]) +
                     A.fd[2] * (sy[2 * BX] - sy[-3 * BX]) + A.fd[3] * (sy[3 * BX] - sy[-4 * BX]);
            }
            if constexpr (NDIM >= 2) {
                Dz = A.fd[0] * (vq[r][4] - vq[r][3]) + A.fd[1] * (vq[r][5] - vq[r][2]) +
                     A.fd[2] * (vq[r][6] - vq[r][1]) + A.fd[3] * (vq[r][7] - vq[r][0]);
            }
            const float S = Dx + Dy + Dz;
            const int L = A.f.cls[g];
            float ps[N];
            load_vec<N>(A.f.psi2 + g * N, ps);
            float Tt = s_ik[L] * S;
#pragma unroll
            for (int nu = 0; nu < N; ++nu) {
                ps[nu] = s_b[nu][L] * ps[nu] + s_a[nu][L] * S;
                Tt += ps[nu];
            }
            store_vec<N>(A.f.psi2 + g * N, ps);
            if (A.pml > 0) {
                const int64_t cc[3] = {x, NDIM == 3 ? yr[r] : z, z};
                const int64_t nn[3] = {nx, NDIM == 3 ? ny : nmarch, nmarch};
                const float Dd[3] = {Dx, NDIM == 3 ? Dy : Dz, Dz};
#pragma unroll
                for (int a = 0; a < NDIM; ++a) {
                    const int64_t c = cc[a], n = nn[a];
                    if (c < A.pml || c >= n - A.pml) {
                        const int32_t off = D.pml_off[a];
                        const float aC = A.pml_tab[off + 2 * n + c];
                        const float bC = A.pml_tab[off + 3 * n + c];
                        float *pp = A.f.pP2[a];
                        const float qv = bC * pp[g] + aC * Dd[a];
                        pp[g] = qv;
                        Tt += qv;
                    }
                }
            }
            float K = s_K[L];
            if (A.noise_amp != 0.0f) {
                const uint64_t li = (uint64_t)(g - base);
                const uint64_t hsh = splitmix64(D.noise_seed ^ li);
                const float u = (float)(hsh >> 40) * 0x1.0p-24f;
                const float e = A.noise_amp * (2.0f * u - 1.0f);
                const float f1 = 1.0f + e;
                K = K * (f1 * f1);
            }
            const float pn = p[g];
            p[g] = pn - A.dt * (K + s_tb[L] * pn) * Tt;
        }
        __syncthreads();
        if constexpr (NDIM >= 2) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
#pragma unroll
                for (int j = 0; j < 7; ++j) vq[r][j] = vq[r][j + 1];
            }
        }
    }
}

// Sources then receivers then the step counter, in one workgroup so the
// receivers see the injected values.
__global__ __launch_bounds__(1024) void k_src_rec(const SrcRecArgs A)
{
    const int64_t t = *A.step;
    if (t < A.n_t) {
        for (int64_t s = threadIdx.x; s < A.n_src; s += blockDim.x)
            A.p[A.src_cell[s]] += A.waves[(int64_t)A.src_wave[s] * A.n_t + t];
    }
    __threadfence();
    __syncthreads();
    if (t < A.n_t_max) {
        for (int64_t r = threadIdx.x; r < A.n_rec; r += blockDim.x)
            A.traces[t * A.n_rec + r] = A.p[A.rec_cell[r]];
    }
    __syncthreads();
    if (threadIdx.x == 0) *A.step = t + 1;
}

template <int NDIM, int N, int BX, int BY, int RY>
hipError_t launch_pair(bool velocity, const StepArgs &a, hipStream_t s)
{
    const dim3 block(BX, BY);
    const dim3 grid(8 * a.tiles_per_xcd);
    if (velocity)
        k_velocity<NDIM, N, BX, BY, RY><<<grid, block, 0, s>>>(a);
    else
        k_pressure<NDIM, N, BX, BY, RY><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

template <int NDIM, int N>
hipError_t launch_nd(bool velocity, int tile_rows, const StepArgs &a, hipStream_t s)
{
    if constexpr (NDIM == 3) {
        if (tile_rows == 8) return launch_pair<3, N, 64, 4, 2>(velocity, a, s);
        return launch_pair<3, N, 64, 4, 4>(velocity, a, s);
    } else if constexpr (NDIM == 2) {
        return launch_pair<2, N, 64, 1, 1>(velocity, a, s);
    } else {
        return launch_pair<1, N, 256, 1, 1>(velocity, a, s);
    }
}

template <int NDIM>
hipError_t launch_n(bool velocity, int nmech, int tile_rows, const StepArgs &a, hipStream_t s)
{
    switch (nmech) {
    case 1: return launch_nd<NDIM, 1>(velocity, tile_rows, a, s);
    case 2: return launch_nd<NDIM, 2>(velocity, tile_rows, a, s);
    case 3: return launch_nd<NDIM, 3>(velocity, tile_rows, a, s);
    case 4: return launch_nd<NDIM, 4>(velocity, tile_rows, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_any(bool velocity, int ndim, int nmech, int tile_rows, const StepArgs &a, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    switch (ndim) {
    case 1: return launch_n<1>(velocity, nmech, tile_rows, a, s);
    case 2: return launch_n<2>(velocity, nmech, tile_rows, a, s);
    case 3: return launch_n<3>(velocity, nmech, tile_rows, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

void tile_shape(int ndim, int tile_rows, int *tx, int *ty)
{
    if (ndim == 3) {
        *tx = 64;
        *ty = tile_rows == 8 ? 8 : 16;
    } else if (ndim == 2) {
        *tx = 64;
        *ty = 1;
    } else {
        *tx = 256;
        *ty = 1;
    }
}

hipError_t launch_velocity(int ndim, int nmech, int tile_rows, const StepArgs &a, hipStream_t s)
{
    return launch_any(true, ndim, nmech, tile_rows, a, s);
}

hipError_t launch_pressure(int ndim, int nmech, int tile_rows, const StepArgs &a, hipStream_t s)
{
    return launch_any(false, ndim, nmech, tile_rows, a, s);
}

hipError_t launch_src_rec(const SrcRecArgs &a, hipStream_t s)
{
    k_src_rec<<<dim3(1), dim3(1024), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace fw
