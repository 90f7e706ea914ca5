// gfx950 kernels of the FDTD step: velocity update, pressure update and the
// source/receiver step.  Paper: Sec. 2.1 (stretched pressure-velocity system,
// memory-variable recursion of Eq. relaxation_psi), Sec. 3.3 (staggered
// stencil of order 8 in space, M = 4).
//
// Work decomposition.  A tile is a 64-cell run along x (times a band of rows
// along y in 3D) that marches along the slowest axis (z in 3D, y in 2D).
// Each thread owns one column per row of the band and keeps the pressure
// (velocity kernel) or the marching-axis velocity (pressure kernel) of eight
// consecutive planes in registers, so the marching-axis stencil costs no
// extra memory traffic.  The x and y stencils read the current plane from a
// double-buffered LDS tile.  The plane after the current one is prefetched
// into registers (own state, queue entry and halo) while the current plane is
// computed, so each plane costs one barrier and HBM latency overlaps the
// arithmetic.  Every output cell is written by exactly one thread with a
// fixed operation order, so results do not depend on the tiling, the batching
// or the launch path.  Blocks are mapped to tiles so that each of the eight
// XCDs receives a contiguous range of the tile list (workgroups are
// dispatched round-robin over the XCDs), keeping neighbouring tiles and their
// halos in one L2.
//
// 3D grids use the plane kernels further down instead (by default):
// short tiles (one plane for the velocity update, two to eight for the
// pressure update) on plane-major lists in which XCD k owns y-band k of every
// plane, with the z stencil read from memory.  2D grids use the 2D tile
// kernels by default: one 64 x R tile per block, both stencils from LDS.  All
// of them compute the same operations in the same order as the marching
// kernels.
#include <algorithm>

#include "fw_internal.h"
#include "fw_vec.h"

namespace fw {

namespace {

// Tile of iteration `it` of this block, or -1.  XCD x (= block % 8, as
// workgroups are dispatched round-robin over the 8 XCDs) owns the contiguous
// tile range [x C, (x + 1) C), C = tiles_per_xcd; its blocks interleave over
// that range with stride blocks_per_xcd (one iteration when the grid has a
// block per tile, several for a persistent grid).
__device__ __forceinline__ int tile_index(const StepArgs &A, int it)
{
    const int b = blockIdx.x;
    const int local = (b >> 3) + it * A.blocks_per_xcd;
    if (local >= A.tiles_per_xcd) return -1;
    const int ti = (b & 7) * A.tiles_per_xcd + local;
    return ti < A.n_tiles ? ti : -1;
}

__device__ __forceinline__ bool in_slab(int64_t c, int64_t n, int P) { return P > 0 && (c < P || c >= n - P); }

// Relaxation strength scale of a cell (1 without a strength map).  With the
// scale the coefficient is s * a; s = 1 reproduces a exactly.
__device__ __forceinline__ float strength(const StepArgs &A, const DomainDesc &D, int u)
{
    return A.amap ? A.amap[D.packed_off + u] : 1.0f;
}

// Per-domain base pointers (uniform over the block, kept in scalar registers)
// so that every per-thread index below is a 32-bit domain-local offset.
struct DomPtrs {
    float *p, *v[3], *psi1[3], *psi2, *pP1[3], *pP2[3];
    const uint8_t *cls;
};

template <int N>
__device__ __forceinline__ DomPtrs dom_ptrs(const Fields &F, const DomainDesc &D)
{
    const int64_t o = D.cell_off;
    DomPtrs d;
    d.p = F.p + o;
    d.v[0] = F.vx + o;
    d.v[1] = F.vy + o;
    d.v[2] = F.vz + o;
    d.psi1[0] = F.psi1x + o * N;
    d.psi1[1] = F.psi1y + o * N;
    d.psi1[2] = F.psi1z + o * N;
    d.psi2 = F.psi2 + o * N;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d.pP1[a] = F.pP1[a] + o;
        d.pP2[a] = F.pP2[a] + o;
    }
    d.cls = F.cls + o;
    return d;
}

// Geometry of a tile as seen by one thread (32-bit domain-local indices).
// Stored index g = col + z * sm (rows px cells apart); the caller's unpadded
// index u = ucol + z * usm (rows nx apart) keys the speed perturbation and
// the strength map.
template <int NDIM, int BX, int BY, int RY>
struct TileGeom {
    int nx, ny, px, nmarch, sm, usm, x;
    int yr[RY], col[RY], ucol[RY];
    bool ok[RY];
    __device__ __forceinline__ void init(const Tile &T, const DomainDesc &D)
    {
        nx = (int)D.n[0];
        ny = (int)D.n[1];
        px = D.pitch;
        nmarch = NDIM == 3 ? (int)D.n[2] : (NDIM == 2 ? (int)D.n[1] : 1);
        sm = NDIM == 3 ? px * ny : px;
        usm = NDIM == 3 ? nx * ny : nx;
        x = T.x0 + (int)threadIdx.x;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            yr[r] = NDIM == 3 ? T.y0 + (int)threadIdx.y * RY + r : 0;
            ok[r] = x < nx && (NDIM < 3 || yr[r] < ny);
            col[r] = (NDIM == 3 ? yr[r] * px : 0) + x;
            ucol[r] = (NDIM == 3 ? yr[r] * nx : 0) + x;
        }
    }
};

// ---------------------------------------------------------------------------
// Velocity update: for each axis a and face i+1/2,
//   D = sum_m c_m (p[i+m] - p[i+1-m]) / dx,
//   psiP    <- bF psiP + aF D,  D <- D + psiP   (inside the CPML slab of a),
//   psi1_nu <- b1_nu psi1_nu + a1_nu D           (class of the owner cell i),
//   v_a     -= 2 dt / (rho_i + rho_{i+1}) (D / kappa_1 + sum_nu psi1_nu).
// The CPML stretch and the tissue stretch are applied one after the other
// (their product is the stretch of the absorbing layer: the layer stretches
// the coordinate of the lossy medium itself); as both are linear recursions
// with fixed coefficients at a point, their order does not matter.
// ---------------------------------------------------------------------------
template <int NDIM, int N, int BX, int BY, int RY>
__global__ __launch_bounds__(BX *BY) void k_velocity(const StepArgs A)
{
    constexpr int TY = NDIM == 3 ? BY * RY : 1;
    constexpr int LX = BX + 8;
    constexpr int LY = NDIM == 3 ? TY + 8 : 1;
    constexpr int NT = BX * BY;
    constexpr int CX = BX + 1;
    constexpr int NHALO = NDIM == 3 ? 8 * LX + 8 * TY : 8;
    constexpr int HS = (NHALO + NT - 1) / NT;
    constexpr int NCH = NDIM == 3 ? TY + BX : 1;
    constexpr int CS = (NCH + NT - 1) / NT;
    constexpr bool MARCH = NDIM >= 2;
    static_assert(NDIM == 3 || (BY == 1 && RY == 1), "bands of rows are 3D only");
    __shared__ float sp[2][LY * LX];
    __shared__ uint8_t scl[2][(TY + 1) * CX];
    // per-class coefficients of this domain, A.class_cap entries per table
    extern __shared__ float s_dyn[];
    const int C = A.class_cap;
    float *s_ik = s_dyn, *s_rho = s_dyn + C, *s_a = s_dyn + 2 * C, *s_b = s_dyn + (2 + N) * C;

    for (int it = 0;; ++it) {
    const int ti = tile_index(A, it);
    if (ti < 0) break;
    if (it > 0) __syncthreads();   // the previous tile is done with the LDS buffers

    const Tile T = A.tiles[ti];
    if (T.z1 <= T.z0) continue;    // padding of a banded tile list
    const DomainDesc D = A.doms[T.dom];
    const int tid = threadIdx.y * BX + threadIdx.x;
    const int tx = threadIdx.x;
    for (int c = tid; c < D.n_classes; c += NT) {
        const ClassCoef &cc = A.classes[D.class_base + c];
        s_ik[c] = cc.ik1;
        s_rho[c] = cc.rho;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            s_a[nu * C + c] = cc.a1[nu];
            s_b[nu * C + c] = cc.b1[nu];
        }
    }
    TileGeom<NDIM, BX, BY, RY> G;
    G.init(T, D);
    // state read from A.f, written to A.fo (the same buffers when stepping in place)
    const DomPtrs M = dom_ptrs<N>(A.f, D);
    const DomPtrs Mo = dom_ptrs<N>(A.fo, D);
    const int P = A.pml;

    // halo slots of this thread: plane-relative offset (-1: outside the
    // domain, value 0) and LDS index (-1: no slot)
    int hoff[HS], hli[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        const int h = tid + s * NT;
        int hy = 0, hx = 0;
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
            hx = h < 4 ? h : BX + h;
        }
        const int gx = T.x0 - 4 + hx;
        const int gy = NDIM == 3 ? T.y0 - 4 + hy : 0;
        const bool inside = gx >= 0 && gx < G.nx && (NDIM < 3 || (gy >= 0 && gy < G.ny));
        hli[s] = h < NHALO ? hy * LX + hx : -1;
        hoff[s] = (h < NHALO && inside) ? (NDIM == 3 ? gy * G.px : 0) + gx : -1;
    }
    int coff[CS], cli[CS];
#pragma unroll
    for (int s = 0; s < CS; ++s) {
        const int h = tid + s * NT;
        int gx, gy, li;
        if (h < TY) {
            gx = T.x0 + BX;
            gy = NDIM == 3 ? T.y0 + h : 0;
            li = h * CX + BX;
        } else {
            gx = T.x0 + (h - TY);
            gy = T.y0 + TY;
            li = TY * CX + (h - TY);
        }
        const bool inside = gx < G.nx && (NDIM < 3 || gy < G.ny);
        cli[s] = h < NCH ? li : -1;
        coff[s] = (h < NCH && inside) ? (NDIM == 3 ? gy * G.px : 0) + gx : -1;
    }

    // registers: pressure queue, class queue, current-plane private state
    float q[RY][8];
    int cq[RY][2];
    float vc[RY][NDIM], pc[RY][NDIM][N], ppc[RY][NDIM];
    const int z0 = T.z0, z1 = T.z1;

    auto coord = [&](int r, int z, int a) { return a == 0 ? G.x : (a == 1 && NDIM == 3 ? G.yr[r] : z); };
    auto extent = [&](int a) { return a == 0 ? G.nx : (a == 1 && NDIM == 3 ? G.ny : G.nmarch); };
    auto load_private = [&](int z, float (&v)[RY][NDIM], float (&ps)[RY][NDIM][N], float (&pp)[RY][NDIM]) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!G.ok[r]) continue;
            const int g = G.col[r] + z * G.sm;
#pragma unroll
            for (int a = 0; a < NDIM; ++a) {
                v[r][a] = M.v[a][g];
                load_stream<N>(M.psi1[a] + (size_t)g * N, ps[r][a]);
                pp[r][a] = in_slab(coord(r, z, a), extent(a), P) ? M.pP1[a][g] : 0.0f;
            }
        }
    };

    // ---- prologue: queue, plane z0 state, LDS buffer 0 ----
#pragma unroll
    for (int r = 0; r < RY; ++r) {
#pragma unroll
        for (int j = 0; j < 8; ++j) q[r][j] = 0.0f;
        cq[r][0] = cq[r][1] = 0;
        if (!G.ok[r]) continue;
        if constexpr (MARCH) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int zz = z0 - 3 + j;
                q[r][j] = (zz >= 0 && zz < G.nmarch) ? M.p[G.col[r] + zz * G.sm] : 0.0f;
            }
            cq[r][0] = M.cls[G.col[r] + z0 * G.sm];
            cq[r][1] = (z0 + 1 < G.nmarch) ? M.cls[G.col[r] + (z0 + 1) * G.sm] : cq[r][0];
        } else {
            q[r][3] = M.p[G.col[r]];
            cq[r][0] = M.cls[G.col[r]];
        }
    }
    load_private(z0, vc, pc, ppc);
    {
        const int zoff = z0 * G.sm;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int row = NDIM == 3 ? threadIdx.y * RY + r : 0;
            sp[0][(NDIM == 3 ? row + 4 : 0) * LX + 4 + tx] = q[r][3];
            scl[0][row * CX + tx] = (uint8_t)cq[r][0];
        }
#pragma unroll
        for (int s = 0; s < HS; ++s)
            if (hli[s] >= 0) sp[0][hli[s]] = hoff[s] >= 0 ? M.p[zoff + hoff[s]] : 0.0f;
#pragma unroll
        for (int s = 0; s < CS; ++s)
            if (cli[s] >= 0) scl[0][cli[s]] = coff[s] >= 0 ? M.cls[zoff + coff[s]] : (uint8_t)0;
    }
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        const bool more = z + 1 < z1;
        // ---- prefetch plane z + 1 ----
        float vn[RY][NDIM], pn[RY][NDIM][N], ppn[RY][NDIM];
        float qn[RY];
        int cqn[RY];
        float hp[HS];
        uint8_t hc[CS];
        if (more) {
            load_private(z + 1, vn, pn, ppn);
            const int zoff = (z + 1) * G.sm;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                qn[r] = 0.0f;
                cqn[r] = cq[r][1];
                if (!G.ok[r]) continue;
                if (z + 5 < G.nmarch) qn[r] = M.p[G.col[r] + (z + 5) * G.sm];
                if (z + 2 < G.nmarch) cqn[r] = M.cls[G.col[r] + (z + 2) * G.sm];
            }
#pragma unroll
            for (int s = 0; s < HS; ++s) hp[s] = hoff[s] >= 0 ? M.p[zoff + hoff[s]] : 0.0f;
#pragma unroll
            for (int s = 0; s < CS; ++s) hc[s] = coff[s] >= 0 ? M.cls[zoff + coff[s]] : (uint8_t)0;
        }

        // ---- compute plane z ----
        const float *spb = sp[b];
        const uint8_t *sclb = scl[b];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!G.ok[r]) continue;
            const int row = NDIM == 3 ? threadIdx.y * RY + r : 0;
            const float *sr = spb + (NDIM == 3 ? row + 4 : 0) * LX + 4 + tx;
            const int g = G.col[r] + z * G.sm;
            const int L = cq[r][0];
            const float ms = strength(A, D, G.ucol[r] + z * G.usm);
            float Dv[3];
            int Ln[3];
            Dv[0] = stencil4(A.fd, sr[1] - sr[0], sr[2] - sr[-1], sr[3] - sr[-2], sr[4] - sr[-3]);
            Ln[0] = (G.x + 1 < G.nx) ? sclb[row * CX + tx + 1] : L;
            if constexpr (NDIM == 3) {
                Dv[1] = stencil4(A.fd, sr[LX] - sr[0], sr[2 * LX] - sr[-LX], sr[3 * LX] - sr[-2 * LX],
                                 sr[4 * LX] - sr[-3 * LX]);
                Ln[1] = (G.yr[r] + 1 < G.ny) ? sclb[(row + 1) * CX + tx] : L;
            }
            if constexpr (MARCH) {
                Dv[NDIM - 1] = stencil4(A.fd, q[r][4] - q[r][3], q[r][5] - q[r][2], q[r][6] - q[r][1],
                                        q[r][7] - q[r][0]);
                Ln[NDIM - 1] = (z + 1 < G.nmarch) ? cq[r][1] : L;
            }
#pragma unroll
            for (int a = 0; a < NDIM; ++a) {
                // CPML stage first (slab cells only): D <- D + psiP, then the
                // tissue stretch of the result; the two stretches compose
                float Da = Dv[a];
                const int c = coord(r, z, a), n = extent(a);
                if (in_slab(c, n, P)) {
                    const int32_t off = D.pml_off[a];
                    const float aF = A.pml_tab[off + c];
                    const float bF = A.pml_tab[off + n + c];
                    const float qv = fmaf(aF, Da, bF * ppc[r][a]);
                    Mo.pP1[a][g] = qv;
                    Da += qv;
                }
                const float m = 2.0f * A.dt / (s_rho[L] + s_rho[Ln[a]]);
                float s = s_ik[L] * Da;
#pragma unroll
                for (int nu = 0; nu < N; ++nu) {
                    pc[r][a][nu] = fmaf(ms * s_a[nu * C + L], Da, s_b[nu * C + L] * pc[r][a][nu]);
                    s += pc[r][a][nu];
                }
                store_stream<N>(Mo.psi1[a] + (size_t)g * N, pc[r][a]);
                store1_stream(Mo.v[a] + g, fmaf(-m, s, vc[r][a]));
            }
        }

        // ---- rotate and stage plane z + 1 ----
        if (more) {
            const int nb = b ^ 1;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                if constexpr (MARCH) {
#pragma unroll
                    for (int j = 0; j < 7; ++j) q[r][j] = q[r][j + 1];
                    q[r][7] = qn[r];
                    cq[r][0] = cq[r][1];
                    cq[r][1] = cqn[r];
                }
#pragma unroll
                for (int a = 0; a < NDIM; ++a) {
                    vc[r][a] = vn[r][a];
                    ppc[r][a] = ppn[r][a];
#pragma unroll
                    for (int nu = 0; nu < N; ++nu) pc[r][a][nu] = pn[r][a][nu];
                }
                const int row = NDIM == 3 ? threadIdx.y * RY + r : 0;
                sp[nb][(NDIM == 3 ? row + 4 : 0) * LX + 4 + tx] = q[r][3];
                scl[nb][row * CX + tx] = (uint8_t)cq[r][0];
            }
#pragma unroll
            for (int s = 0; s < HS; ++s)
                if (hli[s] >= 0) sp[nb][hli[s]] = hp[s];
#pragma unroll
            for (int s = 0; s < CS; ++s)
                if (cli[s] >= 0) scl[nb][cli[s]] = hc[s];
            __syncthreads();
        }
    }
    }  // tile loop
}

// ---------------------------------------------------------------------------
// Pressure update: for each cell,
//   D_a = sum_m c_m (v_a[i+m-1] - v_a[i-m]) / dx,
//   psiP_a  <- bC psiP_a + aC D_a,  D_a <- D_a + psiP_a  (CPML slab of a),
//   S = sum_a D_a,
//   psi2_nu <- b2_nu psi2_nu + a2_nu S     (summed over axes: the tissue
//              coefficients are the same for every axis, so the sum of the
//              per-axis recursions is itself one recursion),
//   p       -= dt (K (1 + eps)^2 + 2 beta p) (S / kappa_2 + sum_nu psi2_nu).
// ---------------------------------------------------------------------------
template <int NDIM, int N, int BX, int BY, int RY>
__global__ __launch_bounds__(BX *BY) void k_pressure(const StepArgs A)
{
    constexpr int TY = NDIM == 3 ? BY * RY : 1;
    constexpr int LX = BX + 8;
    constexpr int LY = NDIM == 3 ? TY + 8 : 1;
    constexpr int NT = BX * BY;
    constexpr int NHALO = 8 * TY + (NDIM == 3 ? 8 * BX : 0);
    constexpr int HS = (NHALO + NT - 1) / NT;
    constexpr bool MARCH = NDIM >= 2;
    static_assert(NDIM == 3 || (BY == 1 && RY == 1), "bands of rows are 3D only");
    __shared__ float svx[2][TY * LX];
    __shared__ float svy[2][NDIM == 3 ? LY * BX : 1];
    extern __shared__ float s_dyn[];
    const int C = A.class_cap;
    float *s_ik = s_dyn, *s_K = s_dyn + C, *s_tb = s_dyn + 2 * C, *s_a = s_dyn + 3 * C, *s_b = s_dyn + (3 + N) * C;

    for (int it = 0;; ++it) {
    const int ti = tile_index(A, it);
    if (ti < 0) break;
    if (it > 0) __syncthreads();   // the previous tile is done with the LDS buffers

    const Tile T = A.tiles[ti];
    if (T.z1 <= T.z0) continue;    // padding of a banded tile list
    const DomainDesc D = A.doms[T.dom];
    const int tid = threadIdx.y * BX + threadIdx.x;
    const int tx = threadIdx.x;
    for (int c = tid; c < D.n_classes; c += NT) {
        const ClassCoef &cc = A.classes[D.class_base + c];
        s_ik[c] = cc.ik2;
        s_K[c] = cc.K;
        s_tb[c] = cc.twobeta;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            s_a[nu * C + c] = cc.a2[nu];
            s_b[nu * C + c] = cc.b2[nu];
        }
    }
    TileGeom<NDIM, BX, BY, RY> G;
    G.init(T, D);
    // p and the memory variables read from A.f, the new velocity and every
    // write in A.fo (the same buffers when stepping in place)
    const DomPtrs M = dom_ptrs<N>(A.f, D);
    const DomPtrs Mo = dom_ptrs<N>(A.fo, D);
    const float *__restrict__ vm = NDIM == 3 ? Mo.v[2] : Mo.v[1];
    const int P = A.pml;

    // halo slots: x-halo of vx (8 per row), then y-halo of vy (8 rows, 3D).
    // hli >= 0 indexes svx, hli <= -2 indexes svy as -(hli + 2), -1: no slot.
    int hoff[HS], hli[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        const int h = tid + s * NT;
        int gx, gy, li;
        if (h < 8 * TY) {
            const int row = h >> 3, k = h & 7;
            const int hx = k < 4 ? k : BX + k;
            gx = T.x0 - 4 + hx;
            gy = NDIM == 3 ? T.y0 + row : 0;
            li = row * LX + hx;
        } else {
            const int hh = h - 8 * TY;
            const int rr = hh / BX;
            const int hy = rr < 4 ? rr : TY + rr;
            const int hx = hh - rr * BX;
            gx = T.x0 + hx;
            gy = T.y0 - 4 + hy;
            li = -(hy * BX + hx) - 2;
        }
        const bool inside = gx >= 0 && gx < G.nx && (NDIM < 3 || (gy >= 0 && gy < G.ny));
        hli[s] = h < NHALO ? li : -1;
        hoff[s] = (h < NHALO && inside) ? (NDIM == 3 ? gy * G.px : 0) + gx : -1;
    }
    auto halo_load = [&](int s, int zoff) -> float {
        if (hoff[s] < 0) return 0.0f;
        return hli[s] >= 0 ? Mo.v[0][zoff + hoff[s]] : Mo.v[1][zoff + hoff[s]];
    };
    auto halo_store = [&](int buf, int s, float val) {
        if (hli[s] >= 0) {
            svx[buf][hli[s]] = val;
        } else if (hli[s] <= -2) {
            if constexpr (NDIM == 3) svy[buf][-(hli[s] + 2)] = val;
        }
    };

    float vq[RY][8];
    float pc[RY], psc[RY][N], ppc[RY][NDIM], vxo[RY], vyo[RY];
    int cc_[RY];
    const int z0 = T.z0, z1 = T.z1;

    auto coord = [&](int r, int z, int a) { return a == 0 ? G.x : (a == 1 && NDIM == 3 ? G.yr[r] : z); };
    auto extent = [&](int a) { return a == 0 ? G.nx : (a == 1 && NDIM == 3 ? G.ny : G.nmarch); };
    auto load_private = [&](int z, float (&pv)[RY], float (&ps)[RY][N], float (&pp)[RY][NDIM], int (&cl)[RY],
                            float (&ox)[RY], float (&oy)[RY]) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            pv[r] = 0.0f;
            cl[r] = 0;
            ox[r] = 0.0f;
            oy[r] = 0.0f;
            if (!G.ok[r]) continue;
            const int g = G.col[r] + z * G.sm;
            pv[r] = M.p[g];
            cl[r] = M.cls[g];
            load_stream<N>(M.psi2 + (size_t)g * N, ps[r]);
            ox[r] = Mo.v[0][g];
            if constexpr (NDIM == 3) oy[r] = Mo.v[1][g];
#pragma unroll
            for (int a = 0; a < NDIM; ++a) pp[r][a] = in_slab(coord(r, z, a), extent(a), P) ? M.pP2[a][g] : 0.0f;
        }
    };
    auto stage = [&](int buf, const float (&ox)[RY], const float (&oy)[RY]) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int row = NDIM == 3 ? threadIdx.y * RY + r : 0;
            svx[buf][row * LX + 4 + tx] = ox[r];
            if constexpr (NDIM == 3) svy[buf][(row + 4) * BX + tx] = oy[r];
        }
    };

    // ---- prologue ----
#pragma unroll
    for (int r = 0; r < RY; ++r) {
#pragma unroll
        for (int j = 0; j < 8; ++j) vq[r][j] = 0.0f;
        if constexpr (MARCH) {
            if (!G.ok[r]) continue;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int zz = z0 - 4 + j;
                vq[r][j] = (zz >= 0 && zz < G.nmarch) ? vm[G.col[r] + zz * G.sm] : 0.0f;
            }
        }
    }
    load_private(z0, pc, psc, ppc, cc_, vxo, vyo);
    stage(0, vxo, vyo);
#pragma unroll
    for (int s = 0; s < HS; ++s) halo_store(0, s, halo_load(s, z0 * G.sm));
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        const bool more = z + 1 < z1;
        float pn[RY], psn[RY][N], ppn[RY][NDIM], vxn[RY], vyn[RY], vqn[RY];
        int cn[RY];
        float hval[HS];
        if (more) {
            load_private(z + 1, pn, psn, ppn, cn, vxn, vyn);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                vqn[r] = 0.0f;
                if (MARCH && G.ok[r] && z + 4 < G.nmarch) vqn[r] = vm[G.col[r] + (z + 4) * G.sm];
            }
#pragma unroll
            for (int s = 0; s < HS; ++s) hval[s] = halo_load(s, (z + 1) * G.sm);
        }

        const float *svxb = svx[b];
        const float *svyb = svy[b];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!G.ok[r]) continue;
            const int row = NDIM == 3 ? threadIdx.y * RY + r : 0;
            const int g = G.col[r] + z * G.sm;
            const float *sx = svxb + row * LX + 4 + tx;
            float Dd[3];
            Dd[0] = stencil4(A.fd, sx[0] - sx[-1], sx[1] - sx[-2], sx[2] - sx[-3], sx[3] - sx[-4]);
            if constexpr (NDIM == 3) {
                const float *sy = svyb + (row + 4) * BX + tx;
                Dd[1] = stencil4(A.fd, sy[0] - sy[-BX], sy[BX] - sy[-2 * BX], sy[2 * BX] - sy[-3 * BX],
                                 sy[3 * BX] - sy[-4 * BX]);
            }
            if constexpr (MARCH) {
                Dd[NDIM - 1] = stencil4(A.fd, vq[r][4] - vq[r][3], vq[r][5] - vq[r][2], vq[r][6] - vq[r][1],
                                        vq[r][7] - vq[r][0]);
            }
            // CPML stage per axis first (slab cells only), then the tissue
            // stretch of the summed divergence (its coefficients do not
            // depend on the axis)
#pragma unroll
            for (int a = 0; a < NDIM; ++a) {
                const int c = coord(r, z, a), n = extent(a);
                if (in_slab(c, n, P)) {
                    const int32_t off = D.pml_off[a];
                    const float aC = A.pml_tab[off + 2 * n + c];
                    const float bC = A.pml_tab[off + 3 * n + c];
                    const float qv = fmaf(aC, Dd[a], bC * ppc[r][a]);
                    Mo.pP2[a][g] = qv;
                    Dd[a] += qv;
                }
            }
            float S = Dd[0];
#pragma unroll
            for (int a = 1; a < NDIM; ++a) S += Dd[a];
            const int L = cc_[r];
            const int u = G.ucol[r] + z * G.usm;
            const float ms = strength(A, D, u);
            float Tt = s_ik[L] * S;
#pragma unroll
            for (int nu = 0; nu < N; ++nu) {
                psc[r][nu] = fmaf(ms * s_a[nu * C + L], S, s_b[nu * C + L] * psc[r][nu]);
                Tt += psc[r][nu];
            }
            store_stream<N>(Mo.psi2 + (size_t)g * N, psc[r]);
            float K = s_K[L];
            if (A.noise_amp != 0.0f) K = K * speed_factor_sq(D.noise_seed, (uint32_t)u, A.noise_amp);
            const float pn0 = pc[r];
            store1_stream(Mo.p + g, fmaf(-(A.dt * fmaf(s_tb[L], pn0, K)), Tt, pn0));
        }

        if (more) {
            const int nb = b ^ 1;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                if constexpr (MARCH) {
#pragma unroll
                    for (int j = 0; j < 7; ++j) vq[r][j] = vq[r][j + 1];
                    vq[r][7] = vqn[r];
                }
                pc[r] = pn[r];
                cc_[r] = cn[r];
#pragma unroll
                for (int nu = 0; nu < N; ++nu) psc[r][nu] = psn[r][nu];
#pragma unroll
                for (int a = 0; a < NDIM; ++a) ppc[r][a] = ppn[r][a];
            }
            stage(nb, vxn, vyn);
#pragma unroll
            for (int s = 0; s < HS; ++s) halo_store(nb, s, hval[s]);
            __syncthreads();
        }
    }
    }  // tile loop
}

// ---------------------------------------------------------------------------
// Plane velocity update (3D, 64 x TY tiles of NP planes (1 or 2), TY = 4
// or 8 rows, one tile per block).  Its tile list is plane-major and XCD k owns y-band k of
// every plane, so all XCDs work on the same few planes: the window of the z
// stencil stays in the last-level cache and is read straight from memory
// instead of being carried in a register queue, and the concurrent tiles
// cover one contiguous stretch of each field.  The x/y stencils read an LDS
// tile.  There is no prefetch state, so more waves fit on a SIMD to hide the
// latency.  Each output is computed with the same operations, in the same
// order, as in k_velocity, so the two give identical bits.
// ---------------------------------------------------------------------------
// Tiles of 2 or 4 planes need about 105 scalar registers, which alone limits
// a SIMD to 7 waves; at N <= 2 their vector registers leave room for 8, so
// the compiler is asked for 8 there (it keeps the extra scalars in vector
// lanes).
template <int N, int NP>
constexpr int kVelocityMinWaves = (NP >= 2 && N <= 2) ? 8 : 1;

template <int N, int TY, int NP, bool SMAP>
__global__ __launch_bounds__(64 * TY) __attribute__((amdgpu_waves_per_eu(kVelocityMinWaves<N, NP>)))
void k_velocity_plane(const StepArgs A)
{
    constexpr int NB = NP > 1 ? 2 : 1;      // LDS buffers
    constexpr int BX = 64, LX = BX + 8, LY = TY + 8, NT = BX * TY, CX = BX + 1;
    // halo cells the stencils read: 3 rows above and 4 below the tile over
    // its own columns, 3 columns left and 4 right over its own rows (LDS row
    // hy holds y0 - 4 + hy, column hx holds x0 - 4 + hx; corners never read)
    constexpr int NHALO = 7 * BX + 7 * TY;
    constexpr int HS = (NHALO + NT - 1) / NT;
    constexpr int NCH = TY + BX;
    __shared__ float sp[NB][LY * LX];
    __shared__ uint8_t scl[NB][(TY + 1) * CX];
    extern __shared__ float s_dyn[];
    const int C = A.class_cap;
    float *s_ik = s_dyn, *s_rho = s_dyn + C, *s_a = s_dyn + 2 * C, *s_b = s_dyn + (2 + N) * C;
    const int b = blockIdx.x;
    const int ti = (b & 7) * A.vtiles_per_xcd + (b >> 3);
    if (ti >= A.n_vtiles) return;
    const Tile T = A.vtiles[ti];
    if (T.z1 <= T.z0) return;      // padding of the banded list
    const DomainDesc D = A.doms[T.dom];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    for (int c = tid; c < D.n_classes; c += NT) {
        const ClassCoef &cc = A.classes[D.class_base + c];
        s_ik[c] = cc.ik1;
        s_rho[c] = cc.rho;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            s_a[nu * C + c] = cc.a1[nu];
            s_b[nu * C + c] = cc.b1[nu];
        }
    }
    const int nx = (int)D.n[0], ny = (int)D.n[1], nz = (int)D.n[2], px = D.pitch, sm = px * ny;
    const int x = T.x0 + tx, y = T.y0 + ty;
    const bool ok = x < nx && y < ny;
    const int col = y * px + x;
    const DomPtrs M = dom_ptrs<N>(A.f, D);
    const DomPtrs Mo = dom_ptrs<N>(A.fo, D);
    const int P = A.pml;
    // the z window first (its reads come from the last-level cache and take
    // longest): p at planes z0 - 3 .. z0 + NP + 3, classes at z0 .. z0 + NP
    float q[NP + 7];
    int cz[NP + 1];
#pragma unroll
    for (int j = 0; j < NP + 7; ++j) {
        const int zz = T.z0 - 3 + j;
        q[j] = (ok && zz >= 0 && zz < nz) ? M.p[col + zz * sm] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j <= NP; ++j) {
        const int zz = T.z0 + j;
        cz[j] = (ok && zz < nz) ? M.cls[col + zz * sm] : 0;
    }
    int hoff[HS], hli[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        const int h = tid + s * NT;
        int hy = 0, hx = 0;
        if (h < 7 * BX) {
            const int rr = h / BX;
            hy = rr < 3 ? rr + 1 : TY + 1 + rr;
            hx = 4 + h - rr * BX;
        } else {
            const int hh = h - 7 * BX;
            hy = 4 + hh / 7;
            const int k = hh - (hh / 7) * 7;
            hx = k < 3 ? k + 1 : BX + 1 + k;
        }
        const int gx = T.x0 - 4 + hx, gy = T.y0 - 4 + hy;
        const bool inside = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        hli[s] = h < NHALO ? hy * LX + hx : -1;
        hoff[s] = (h < NHALO && inside) ? gy * px + gx : -1;
    }
    int coff = -1, cli = -1;
    if (tid < NCH) {
        int gx, gy;
        if (tid < TY) {
            gx = T.x0 + BX;
            gy = T.y0 + tid;
            cli = tid * CX + BX;
        } else {
            gx = T.x0 + (tid - TY);
            gy = T.y0 + TY;
            cli = TY * CX + (tid - TY);
        }
        coff = (gx < nx && gy < ny) ? gy * px + gx : -1;
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int z = T.z0 + j;
        if (z >= T.z1) break;
        const int zoff = z * sm;
        const int g = zoff + col;
        float *bp = sp[j % NB];
        uint8_t *bc = scl[j % NB];
#pragma unroll
        for (int s = 0; s < HS; ++s)
            if (hli[s] >= 0) bp[hli[s]] = hoff[s] >= 0 ? M.p[zoff + hoff[s]] : 0.0f;
        if (cli >= 0) bc[cli] = coff >= 0 ? M.cls[zoff + coff] : (uint8_t)0;
        float vc[3], pc[3][N], ppc[3];
        if (ok) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int c = a == 0 ? x : (a == 1 ? y : z), n = a == 0 ? nx : (a == 1 ? ny : nz);
                vc[a] = load1_stream(M.v[a] + g);
                load_stream<N>(M.psi1[a] + (size_t)g * N, pc[a]);
                ppc[a] = in_slab(c, n, P) ? M.pP1[a][g] : 0.0f;
            }
        }
        bp[(ty + 4) * LX + 4 + tx] = q[j + 3];
        bc[ty * CX + tx] = (uint8_t)cz[j];
        // with two buffers, the one written here was last read in plane
        // j - 2, before the barrier of plane j - 1 that every thread passed
        __syncthreads();
        if (!ok) continue;
        const int L = cz[j];
        // strength map (a separate instantiation), keyed by the unpadded index
        const float ms = SMAP ? A.amap[D.packed_off + (int64_t)(z * ny + y) * nx + x] : 1.0f;
        const float *sr = bp + (ty + 4) * LX + 4 + tx;
        float Dv[3];
        int Ln[3];
        Dv[0] = stencil4(A.fd, sr[1] - sr[0], sr[2] - sr[-1], sr[3] - sr[-2], sr[4] - sr[-3]);
        Ln[0] = (x + 1 < nx) ? bc[ty * CX + tx + 1] : L;
        Dv[1] = stencil4(A.fd, sr[LX] - sr[0], sr[2 * LX] - sr[-LX], sr[3 * LX] - sr[-2 * LX], sr[4 * LX] - sr[-3 * LX]);
        Ln[1] = (y + 1 < ny) ? bc[(ty + 1) * CX + tx] : L;
        Dv[2] = stencil4(A.fd, q[j + 4] - q[j + 3], q[j + 5] - q[j + 2], q[j + 6] - q[j + 1], q[j + 7] - q[j]);
        Ln[2] = (z + 1 < nz) ? cz[j + 1] : L;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float Da = Dv[a];
            const int c = a == 0 ? x : (a == 1 ? y : z), n = a == 0 ? nx : (a == 1 ? ny : nz);
            if (in_slab(c, n, P)) {
                const int32_t off = D.pml_off[a];
                const float aF = A.pml_tab[off + c];
                const float bF = A.pml_tab[off + n + c];
                const float qv = fmaf(aF, Da, bF * ppc[a]);
                Mo.pP1[a][g] = qv;
                Da += qv;
            }
            const float m = 2.0f * A.dt / (s_rho[L] + s_rho[Ln[a]]);
            float sacc = s_ik[L] * Da;
#pragma unroll
            for (int nu = 0; nu < N; ++nu) {
                pc[a][nu] = fmaf(ms * s_a[nu * C + L], Da, s_b[nu * C + L] * pc[a][nu]);
                sacc += pc[a][nu];
            }
            store_stream<N>(Mo.psi1[a] + (size_t)g * N, pc[a]);
            store1_stream(Mo.v[a] + g, fmaf(-m, sacc, vc[a]));
        }
    }
}

// Pressure update on tiles of NP consecutive planes (2, 4 or 8; 3D, 64 x TY
// with TY = 4 or 8 rows, one tile per block), from a list in which XCD k owns y-band k of every
// group of planes.  The v_z window of the current plane (planes - 4 .. + 3)
// is carried in registers as a queue: seven planes are loaded before the
// first plane and the eighth with each plane's own operands.  Each plane
// loads the x-halo of v_x, the y-halo of v_y and its own state into
// registers and stages the halos in a double-buffered LDS tile.  The barrier of a plane orders LDS
// only (the threads exchange nothing through global memory), so the loads
// of the next plane, issued right after it, stay in flight while the
// current plane is computed.  Same operations in the same order as
// k_pressure.
// Asking the compiler for 8 waves per SIMD where that fits without scratch
// spills (2-plane tiles, and N <= 2): 6.64 against 6.69 ms at N = 4 and 5.08
// against 5.21 ms at N = 2 on 960 x 960 x 720; the 4- and 8-plane tiles at
// N >= 3 would spill and run slower (7.4-7.5 ms), so they keep 7.
template <int N, int NP>
constexpr int kPressureMinWaves = (NP == 2 || N <= 2) ? 8 : 1;

template <int N, int TY, int NP, bool SMAP>
__global__ __launch_bounds__(64 * TY) __attribute__((amdgpu_waves_per_eu(kPressureMinWaves<N, NP>)))
void k_pressure_planes(const StepArgs A)
{
    constexpr int BX = 64, LX = BX + 8, LY = TY + 8, NT = BX * TY;
    // halo cells the stencils read: x-4 .. x-1 and x+64 .. x+66 of v_x over
    // the tile's rows, y-4 .. y-1 and y+4 .. y+6 of v_y over its columns
    constexpr int NHALO = 7 * TY + 7 * BX;
    constexpr int HS = (NHALO + NT - 1) / NT;
    __shared__ float svx[2][TY * LX];
    __shared__ float svy[2][LY * BX];
    extern __shared__ float s_dyn[];
    const int C = A.class_cap;
    float *s_ik = s_dyn, *s_K = s_dyn + C, *s_tb = s_dyn + 2 * C, *s_a = s_dyn + 3 * C, *s_b = s_dyn + (3 + N) * C;

    const int b = blockIdx.x;
    const int ti = (b & 7) * A.ptiles_per_xcd + (b >> 3);
    if (ti >= A.n_ptiles) return;
    const Tile T = A.ptiles[ti];
    if (T.z1 <= T.z0) return;      // padding of the banded list
    const DomainDesc D = A.doms[T.dom];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    for (int c = tid; c < D.n_classes; c += NT) {
        const ClassCoef &cc = A.classes[D.class_base + c];
        s_ik[c] = cc.ik2;
        s_K[c] = cc.K;
        s_tb[c] = cc.twobeta;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            s_a[nu * C + c] = cc.a2[nu];
            s_b[nu * C + c] = cc.b2[nu];
        }
    }
    const int nx = (int)D.n[0], ny = (int)D.n[1], nz = (int)D.n[2], px = D.pitch, sm = px * ny;
    const int x = T.x0 + tx, y = T.y0 + ty;
    const bool ok = x < nx && y < ny;
    // p and the memory variables read from A.f, the new velocity and every
    // write in A.fo (the same buffers when stepping in place)
    const DomPtrs M = dom_ptrs<N>(A.f, D);
    const DomPtrs Mo = dom_ptrs<N>(A.fo, D);
    const int P = A.pml;
    const int col = y * px + x;

    // v_z of the group's window: planes z0 - 4 .. z0 + NP + 2, zero outside
    float vq[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int zz = T.z0 - 4 + j;
        vq[j] = (ok && zz >= 0 && zz < nz) ? Mo.v[2][col + zz * sm] : 0.0f;
    }
    // halo slots: plane-relative offset (-1: outside the domain, value 0) and
    // target (>= 0: svx index, <= -2: svy index -(li + 2), -1: no slot)
    int hoff[HS], hli[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        const int h = tid + s * NT;
        int gx, gy, li;
        if (h < 7 * TY) {
            const int row = h / 7, k = h - (h / 7) * 7;
            const int hx = k < 4 ? k : BX + k;
            gx = T.x0 - 4 + hx;
            gy = T.y0 + row;
            li = row * LX + hx;
        } else {
            const int hh = h - 7 * TY;
            const int rr = hh / BX;
            const int hy = rr < 4 ? rr : TY + rr;
            const int hx = hh - rr * BX;
            gx = T.x0 + hx;
            gy = T.y0 - 4 + hy;
            li = -(hy * BX + hx) - 2;
        }
        const bool inside = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        hli[s] = h < NHALO ? li : -1;
        hoff[s] = (h < NHALO && inside) ? gy * px + gx : -1;
    }

    // per plane: the halo share and own v_x, v_y first (the LDS staging
    // waits for them only), then the streamed state
    struct PlaneIn {
        float hv[HS], ox, oy, pc, psc[N], ppc[3], vzt;
        int L;
    };
    auto load_plane = [&](int z, PlaneIn &o) {
        const int zoff = z * sm;
        const int g = zoff + col;
        // top of plane z's v_z window (plane z + 3); the rest is carried over
        o.vzt = (ok && z + 3 < nz) ? Mo.v[2][col + (z + 3) * sm] : 0.0f;
#pragma unroll
        for (int s = 0; s < HS; ++s)
            o.hv[s] = (hli[s] == -1 || hoff[s] < 0) ? 0.0f
                      : (hli[s] >= 0 ? Mo.v[0][zoff + hoff[s]] : Mo.v[1][zoff + hoff[s]]);
        o.ox = ok ? Mo.v[0][g] : 0.0f;
        o.oy = ok ? Mo.v[1][g] : 0.0f;
        o.pc = ok ? load1_stream(M.p + g) : 0.0f;
        o.L = ok ? (int)M.cls[g] : 0;
        if (ok)
            load_stream<N>(M.psi2 + (size_t)g * N, o.psc);
        else
#pragma unroll
            for (int nu = 0; nu < N; ++nu) o.psc[nu] = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int c = a == 0 ? x : (a == 1 ? y : z), n = a == 0 ? nx : (a == 1 ? ny : nz);
            o.ppc[a] = (ok && in_slab(c, n, P)) ? M.pP2[a][g] : 0.0f;
        }
    };
    PlaneIn cur, nxt;
    load_plane(T.z0, cur);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int z = T.z0 + j;
        if (z >= T.z1) break;
        const int g = z * sm + col;
        float *bx = svx[j & 1], *by = svy[j & 1];
#pragma unroll
        for (int s = 0; s < HS; ++s) {
            if (hli[s] >= 0)
                bx[hli[s]] = cur.hv[s];
            else if (hli[s] <= -2)
                by[-(hli[s] + 2)] = cur.hv[s];
        }
        bx[ty * LX + 4 + tx] = cur.ox;
        by[(ty + 4) * BX + tx] = cur.oy;
        // LDS-only barrier: the loads in flight keep going.  The buffer
        // written here was last read in plane j - 2, before every thread
        // passed the barrier of plane j - 1
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (j + 1 < NP && z + 1 < T.z1) load_plane(z + 1, nxt);
        if (ok) {   // threads outside the domain still own halo slots
            const float *sx = bx + ty * LX + 4 + tx;
            const float *sy = by + (ty + 4) * BX + tx;
            float Dd[3];
            Dd[0] = stencil4(A.fd, sx[0] - sx[-1], sx[1] - sx[-2], sx[2] - sx[-3], sx[3] - sx[-4]);
            Dd[1] = stencil4(A.fd, sy[0] - sy[-BX], sy[BX] - sy[-2 * BX], sy[2 * BX] - sy[-3 * BX],
                             sy[3 * BX] - sy[-4 * BX]);
            Dd[2] = stencil4(A.fd, vq[4] - vq[3], vq[5] - vq[2], vq[6] - vq[1], cur.vzt - vq[0]);
            const int L = cur.L;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int c = a == 0 ? x : (a == 1 ? y : z), n = a == 0 ? nx : (a == 1 ? ny : nz);
                if (in_slab(c, n, P)) {
                    const int32_t off = D.pml_off[a];
                    const float aC = A.pml_tab[off + 2 * n + c];
                    const float bC = A.pml_tab[off + 3 * n + c];
                    const float qv = fmaf(aC, Dd[a], bC * cur.ppc[a]);
                    Mo.pP2[a][g] = qv;
                    Dd[a] += qv;
                }
            }
            float S = Dd[0];
#pragma unroll
            for (int a = 1; a < 3; ++a) S += Dd[a];
            float Tt = s_ik[L] * S;
            float psn[N];
            // strength map (a separate instantiation): read here rather than
            // with the prefetched state; speed perturbation and map are keyed
            // by the unpadded index
            const int u = (z * ny + y) * nx + x;
            const float ms = SMAP ? A.amap[D.packed_off + u] : 1.0f;
#pragma unroll
            for (int nu = 0; nu < N; ++nu) {
                psn[nu] = fmaf(ms * s_a[nu * C + L], S, s_b[nu * C + L] * cur.psc[nu]);
                Tt += psn[nu];
            }
            store_stream<N>(Mo.psi2 + (size_t)g * N, psn);
            float K = s_K[L];
            if (A.noise_amp != 0.0f) K = K * speed_factor_sq(D.noise_seed, (uint32_t)u, A.noise_amp);
            const float pn0 = cur.pc;
            store1_stream(Mo.p + g, fmaf(-(A.dt * fmaf(s_tb[L], pn0, K)), Tt, pn0));
        }
        // advance the window: planes z - 3 .. z + 3 kept, z + 4 arrives with nxt
#pragma unroll
        for (int i = 0; i < 6; ++i) vq[i] = vq[i + 1];
        vq[6] = cur.vzt;
        cur = nxt;
    }
}

// ---------------------------------------------------------------------------
// 2D tile kernels: one 64 x TY tile of a 2D grid per block (TY = 4, 8 or 16
// rows, one cell per thread), from a list in which XCD k owns y-band k of
// every domain.  Both stencils read an LDS tile holding the halo cells they
// use, so a thread keeps only its own cell's state: no register queue and no
// prefetched row, which leaves room for about twice the waves per SIMD of the
// marching kernels.  The halo rows are rows of the neighbouring tiles of the
// same band, read again from L2.  Same operations in the same order as
// k_velocity / k_pressure in 2D, so the results are identical.
// WIDE: the widened stencil of the fourth-order-in-time set, which adds to
// each axis's difference b times the two-point differences along that axis
// in the rows one cell away on the other axis (both sides); its extra
// operands come from the same LDS tiles, enlarged by one row or column.
// ---------------------------------------------------------------------------
template <int N, int TY, bool SMAP, bool WIDE>
__global__ __launch_bounds__(64 * TY) void k_velocity_tile2d(const StepArgs A)
{
    constexpr int BX = 64, LX = BX + 8, LY = TY + 8, NT = BX * TY, CX = BX + 1;
    // p halo the stencils read: 3 rows above and 4 below the tile over its
    // columns, 3 columns left and 4 right over its rows (LDS row hy holds
    // y0 - 4 + hy, column hx holds x0 - 4 + hx); WIDE also reads the corner
    // cells (x0 + 64, y0 - 1), (x0 + 64, y0 + TY) and (x0 - 1, y0 + TY)
    constexpr int NCORE = 7 * BX + 7 * TY;
    constexpr int NHALO = NCORE + (WIDE ? 3 : 0);
    constexpr int HS = (NHALO + NT - 1) / NT;
    constexpr int NCH = TY + BX;
    __shared__ float sp[LY * LX];
    __shared__ uint8_t scl[(TY + 1) * CX];
    extern __shared__ float s_dyn[];
    const int C = A.class_cap;
    float *s_ik = s_dyn, *s_rho = s_dyn + C, *s_a = s_dyn + 2 * C, *s_b = s_dyn + (2 + N) * C;
    const int b = blockIdx.x;
    const int ti = (b & 7) * A.vtiles_per_xcd + (b >> 3);
    if (ti >= A.n_vtiles) return;
    const Tile T = A.vtiles[ti];
    if (T.z1 <= T.z0) return;      // padding of the banded list
    const DomainDesc D = A.doms[T.dom];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    for (int c = tid; c < D.n_classes; c += NT) {
        const ClassCoef &cc = A.classes[D.class_base + c];
        s_ik[c] = cc.ik1;
        s_rho[c] = cc.rho;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            s_a[nu * C + c] = cc.a1[nu];
            s_b[nu * C + c] = cc.b1[nu];
        }
    }
    const int nx = (int)D.n[0], ny = (int)D.n[1], px = D.pitch;
    const int x = T.x0 + tx, y = T.y0 + ty;
    const bool ok = x < nx && y < ny;
    const int g = y * px + x;
    const DomPtrs M = dom_ptrs<N>(A.f, D);
    const DomPtrs Mo = dom_ptrs<N>(A.fo, D);
    const int P = A.pml;
    // the tile's p and classes, and the halo
    const float p0 = ok ? M.p[g] : 0.0f;
    const int L0 = ok ? (int)M.cls[g] : 0;
    float hv[HS];
    int hli[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        const int h = tid + s * NT;
        int hy = 0, hx = 0;
        if (h < 7 * BX) {
            const int rr = h / BX;
            hy = rr < 3 ? rr + 1 : TY + 1 + rr;
            hx = 4 + h - rr * BX;
        } else if (h < NCORE) {
            const int hh = h - 7 * BX;
            hy = 4 + hh / 7;
            const int k = hh - (hh / 7) * 7;
            hx = k < 3 ? k + 1 : BX + 1 + k;
        } else {
            const int k = h - NCORE;       // WIDE corners (h < NHALO is checked below)
            hx = k == 2 ? 3 : BX + 4;
            hy = k == 0 ? 3 : TY + 4;
        }
        const int gx = T.x0 - 4 + hx, gy = T.y0 - 4 + hy;
        const bool inside = h < NHALO && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        hli[s] = h < NHALO ? hy * LX + hx : -1;
        hv[s] = inside ? M.p[gy * px + gx] : 0.0f;
    }
    int cli = -1;
    uint8_t cv = 0;
    if (tid < NCH) {
        int gx, gy;
        if (tid < TY) {
            gx = T.x0 + BX;
            gy = T.y0 + tid;
            cli = tid * CX + BX;
        } else {
            gx = T.x0 + (tid - TY);
            gy = T.y0 + TY;
            cli = TY * CX + (tid - TY);
        }
        if (gx < nx && gy < ny) cv = M.cls[gy * px + gx];
    }
    // the cell's own streamed state
    float vc[2], pc[2][N], ppc[2];
    if (ok) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int c = a == 0 ? x : y, n = a == 0 ? nx : ny;
            vc[a] = load1_stream(M.v[a] + g);
            load_stream<N>(M.psi1[a] + (size_t)g * N, pc[a]);
            ppc[a] = in_slab(c, n, P) ? M.pP1[a][g] : 0.0f;
        }
    }
    sp[(ty + 4) * LX + 4 + tx] = p0;
    scl[ty * CX + tx] = (uint8_t)L0;
#pragma unroll
    for (int s = 0; s < HS; ++s)
        if (hli[s] >= 0) sp[hli[s]] = hv[s];
    if (cli >= 0) scl[cli] = cv;
    __syncthreads();
    if (!ok) return;
    const int L = L0;
    const float ms = SMAP ? A.amap[D.packed_off + y * nx + x] : 1.0f;
    const float *sr = sp + (ty + 4) * LX + 4 + tx;
    float Dv[2];
    int Ln[2];
    Dv[0] = stencil4(A.fd, sr[1] - sr[0], sr[2] - sr[-1], sr[3] - sr[-2], sr[4] - sr[-3]);
    Ln[0] = (x + 1 < nx) ? scl[ty * CX + tx + 1] : L;
    Dv[1] = stencil4(A.fd, sr[LX] - sr[0], sr[2 * LX] - sr[-LX], sr[3 * LX] - sr[-2 * LX], sr[4 * LX] - sr[-3 * LX]);
    Ln[1] = (y + 1 < ny) ? scl[(ty + 1) * CX + tx] : L;
    if constexpr (WIDE) {
        // face (x + 1/2, y): rows y + 1 and y - 1; face (x, y + 1/2): columns x + 1 and x - 1
        Dv[0] = fmaf(A.fd_b, (sr[LX + 1] - sr[LX]) + (sr[1 - LX] - sr[-LX]), Dv[0]);
        Dv[1] = fmaf(A.fd_b, (sr[LX + 1] - sr[1]) + (sr[LX - 1] - sr[-1]), Dv[1]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        float Da = Dv[a];
        const int c = a == 0 ? x : y, n = a == 0 ? nx : ny;
        if (in_slab(c, n, P)) {
            const int32_t off = D.pml_off[a];
            const float aF = A.pml_tab[off + c];
            const float bF = A.pml_tab[off + n + c];
            const float qv = fmaf(aF, Da, bF * ppc[a]);
            Mo.pP1[a][g] = qv;
            Da += qv;
        }
        const float m = 2.0f * A.dt / (s_rho[L] + s_rho[Ln[a]]);
        float sacc = s_ik[L] * Da;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            pc[a][nu] = fmaf(ms * s_a[nu * C + L], Da, s_b[nu * C + L] * pc[a][nu]);
            sacc += pc[a][nu];
        }
        store_stream<N>(Mo.psi1[a] + (size_t)g * N, pc[a]);
        store1_stream(Mo.v[a] + g, fmaf(-m, sacc, vc[a]));
    }
}

template <int N, int TY, bool SMAP, bool WIDE>
__global__ __launch_bounds__(64 * TY) void k_pressure_tile2d(const StepArgs A)
{
    constexpr int BX = 64, LX = BX + 8, LY = TY + 8, NT = BX * TY;
    // halo cells the stencils read: x-4 .. x-1 and x+64 .. x+66 of v_x over
    // the tile's rows, y-4 .. y-1 and y+TY .. y+TY+2 of v_y over its columns;
    // WIDE also reads v_x in rows y0-1 and y0+TY over columns x0-1 .. x0+63
    // (svx gets a row above and below) and v_y in columns x0-1 and x0+64 over
    // rows y0-1 .. y0+TY-1 (svy gets a column on each side)
    constexpr int RX0 = WIDE ? 1 : 0, SXR = TY + 2 * RX0;     // svx: first tile row, rows
    constexpr int CY0 = WIDE ? 1 : 0, SYC = BX + 2 * CY0;     // svy: first tile column, row pitch
    constexpr int NCORE = 7 * TY + 7 * BX;
    constexpr int NXR = 2 * (BX + 1), NYC = 2 * (TY + 1);     // WIDE extra v_x and v_y cells
    constexpr int NHALO = NCORE + (WIDE ? NXR + NYC : 0);
    constexpr int HS = (NHALO + NT - 1) / NT;
    __shared__ float svx[SXR * LX];
    __shared__ float svy[LY * SYC];
    extern __shared__ float s_dyn[];
    const int C = A.class_cap;
    float *s_ik = s_dyn, *s_K = s_dyn + C, *s_tb = s_dyn + 2 * C, *s_a = s_dyn + 3 * C, *s_b = s_dyn + (3 + N) * C;
    const int b = blockIdx.x;
    const int ti = (b & 7) * A.ptiles_per_xcd + (b >> 3);
    if (ti >= A.n_ptiles) return;
    const Tile T = A.ptiles[ti];
    if (T.z1 <= T.z0) return;      // padding of the banded list
    const DomainDesc D = A.doms[T.dom];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    for (int c = tid; c < D.n_classes; c += NT) {
        const ClassCoef &cc = A.classes[D.class_base + c];
        s_ik[c] = cc.ik2;
        s_K[c] = cc.K;
        s_tb[c] = cc.twobeta;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            s_a[nu * C + c] = cc.a2[nu];
            s_b[nu * C + c] = cc.b2[nu];
        }
    }
    const int nx = (int)D.n[0], ny = (int)D.n[1], px = D.pitch;
    const int x = T.x0 + tx, y = T.y0 + ty;
    const bool ok = x < nx && y < ny;
    const int g = y * px + x;
    // p and the memory variables read from A.f, the new velocity and every
    // write in A.fo (the same buffers when stepping in place)
    const DomPtrs M = dom_ptrs<N>(A.f, D);
    const DomPtrs Mo = dom_ptrs<N>(A.fo, D);
    const int P = A.pml;
    const float ox = ok ? Mo.v[0][g] : 0.0f;
    const float oy = ok ? Mo.v[1][g] : 0.0f;
    // halo: target >= 0 an svx index, <= -2 the svy index -(li + 2), -1 none
    float hv[HS];
    int hli[HS];
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        const int h = tid + s * NT;
        int gx, gy, li;
        if (h < 7 * TY) {
            const int row = h / 7, k = h - (h / 7) * 7;
            const int hx = k < 4 ? k : BX + k;
            gx = T.x0 - 4 + hx;
            gy = T.y0 + row;
            li = (row + RX0) * LX + hx;
        } else if (h < NCORE) {
            const int hh = h - 7 * TY;
            const int rr = hh / BX;
            const int hy = rr < 4 ? rr : TY + rr;
            const int hx = hh - rr * BX;
            gx = T.x0 + hx;
            gy = T.y0 - 4 + hy;
            li = -(hy * SYC + CY0 + hx) - 2;
        } else if (h < NCORE + NXR) {
            // WIDE: v_x of row y0 - 1 (svx row 0) or y0 + TY (svx row TY + 1)
            const int e = h - NCORE, side = e / (BX + 1), hx = 3 + e - side * (BX + 1);
            gx = T.x0 - 4 + hx;
            gy = side == 0 ? T.y0 - 1 : T.y0 + TY;
            li = (side == 0 ? 0 : TY + 1) * LX + hx;
        } else {
            // WIDE: v_y of column x0 - 1 (svy column 0) or x0 + 64 (column BX + 1)
            // (h < NHALO is checked below)
            const int e = h - NCORE - NXR, side = e / (TY + 1), hy = 3 + e - side * (TY + 1);
            gx = side == 0 ? T.x0 - 1 : T.x0 + BX;
            gy = T.y0 - 4 + hy;
            li = -(hy * SYC + (side == 0 ? 0 : BX + 1)) - 2;
        }
        const bool inside = h < NHALO && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        hli[s] = h < NHALO ? li : -1;
        hv[s] = inside ? (li >= 0 ? Mo.v[0][gy * px + gx] : Mo.v[1][gy * px + gx]) : 0.0f;
    }
    // the cell's own streamed state
    float pc = 0.0f, psc[N], ppc[2];
    int L = 0;
    if (ok) {
        pc = load1_stream(M.p + g);
        L = M.cls[g];
        load_stream<N>(M.psi2 + (size_t)g * N, psc);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int c = a == 0 ? x : y, n = a == 0 ? nx : ny;
            ppc[a] = in_slab(c, n, P) ? M.pP2[a][g] : 0.0f;
        }
    }
    svx[(ty + RX0) * LX + 4 + tx] = ox;
    svy[(ty + 4) * SYC + CY0 + tx] = oy;
#pragma unroll
    for (int s = 0; s < HS; ++s) {
        if (hli[s] >= 0)
            svx[hli[s]] = hv[s];
        else if (hli[s] <= -2)
            svy[-(hli[s] + 2)] = hv[s];
    }
    __syncthreads();
    if (!ok) return;
    const float *sx = svx + (ty + RX0) * LX + 4 + tx;
    const float *sy = svy + (ty + 4) * SYC + CY0 + tx;
    float Dd[2];
    Dd[0] = stencil4(A.fd, sx[0] - sx[-1], sx[1] - sx[-2], sx[2] - sx[-3], sx[3] - sx[-4]);
    Dd[1] = stencil4(A.fd, sy[0] - sy[-SYC], sy[SYC] - sy[-2 * SYC], sy[2 * SYC] - sy[-3 * SYC],
                     sy[3 * SYC] - sy[-4 * SYC]);
    if constexpr (WIDE) {
        // cell (x, y): v_x differences in rows y + 1 and y - 1, v_y differences in columns x + 1 and x - 1
        Dd[0] = fmaf(A.fd_b, (sx[LX] - sx[LX - 1]) + (sx[-LX] - sx[-LX - 1]), Dd[0]);
        Dd[1] = fmaf(A.fd_b, (sy[1] - sy[1 - SYC]) + (sy[-1] - sy[-1 - SYC]), Dd[1]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int c = a == 0 ? x : y, n = a == 0 ? nx : ny;
        if (in_slab(c, n, P)) {
            const int32_t off = D.pml_off[a];
            const float aC = A.pml_tab[off + 2 * n + c];
            const float bC = A.pml_tab[off + 3 * n + c];
            const float qv = fmaf(aC, Dd[a], bC * ppc[a]);
            Mo.pP2[a][g] = qv;
            Dd[a] += qv;
        }
    }
    const float S = Dd[0] + Dd[1];
    float Tt = s_ik[L] * S;
    const int u = y * nx + x;
    const float ms = SMAP ? A.amap[D.packed_off + u] : 1.0f;
#pragma unroll
    for (int nu = 0; nu < N; ++nu) {
        psc[nu] = fmaf(ms * s_a[nu * C + L], S, s_b[nu * C + L] * psc[nu]);
        Tt += psc[nu];
    }
    store_stream<N>(Mo.psi2 + (size_t)g * N, psc);
    float K = s_K[L];
    if (A.noise_amp != 0.0f) K = K * speed_factor_sq(D.noise_seed, (uint32_t)u, A.noise_amp);
    store1_stream(Mo.p + g, fmaf(-(A.dt * fmaf(s_tb[L], pc, K)), Tt, pc));
}

// Sources, receivers and the step counter.  One thread per distinct
// source/receiver cell reads p once, adds the cell's source and records the
// result for the cell's receivers, so the receivers see the injected value
// without a second pass.  The last workgroup to finish advances the step
// counter (every workgroup has read it by then) and re-arms the count.
__global__ __launch_bounds__(256) void k_src_rec(const SrcRecArgs A)
{
    __shared__ int s_last;
    const int64_t t = *A.step;
    const bool inject = t < A.n_t, record = t < A.n_t_max;
    bool bad = false;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < A.n_cells) {
        const SrcRecCell c = A.cells[e];
        float v = A.p[c.cell];
        if (inject && c.wave >= 0) {
            v += A.waves[(int64_t)c.wave * A.n_t + t];
            A.p[c.cell] = v;
        }
        if (record) {
            for (int32_t k = c.r0; k < c.r1; ++k) A.traces[t * A.n_rec + A.rec_of[k]] = v;
            bad = c.r1 > c.r0 && !isfinite(v);
        }
    }
    // finite check: every thread that saw a non-finite value writes the same
    // row, and only while no earlier row has been flagged
    if (bad && *A.bad_row < 0) *A.bad_row = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(A.done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        *A.done = 0u;
        *A.step = t + 1;
    }
}

template <int NDIM, int N, int BX, int BY, int RY>
hipError_t launch_pair(bool velocity, const StepArgs &a, hipStream_t s)
{
    const dim3 block(BX, BY);
    const dim3 grid(8 * a.blocks_per_xcd);
    const size_t lds = (size_t)a.class_cap * (velocity ? 2 + 2 * N : 3 + 2 * N) * sizeof(float);
    if (velocity)
        k_velocity<NDIM, N, BX, BY, RY><<<grid, block, lds, s>>>(a);
    else
        k_pressure<NDIM, N, BX, BY, RY><<<grid, block, lds, s>>>(a);
    return hipGetLastError();
}

// plane kernels: tile rows (4 or 8) x planes per tile
template <int N, bool SMAP>
hipError_t launch_velocity_plane(const StepArgs &a, size_t lds, hipStream_t s)
{
    const dim3 grid(8 * a.vtiles_per_xcd);
    if (a.plane_rows == 8) {
        if (a.vel_planes == 4)
            k_velocity_plane<N, 8, 4, SMAP><<<grid, dim3(64, 8), lds, s>>>(a);
        else if (a.vel_planes == 2)
            k_velocity_plane<N, 8, 2, SMAP><<<grid, dim3(64, 8), lds, s>>>(a);
        else
            k_velocity_plane<N, 8, 1, SMAP><<<grid, dim3(64, 8), lds, s>>>(a);
    } else {
        if (a.vel_planes == 4)
            k_velocity_plane<N, 4, 4, SMAP><<<grid, dim3(64, 4), lds, s>>>(a);
        else if (a.vel_planes == 2)
            k_velocity_plane<N, 4, 2, SMAP><<<grid, dim3(64, 4), lds, s>>>(a);
        else
            k_velocity_plane<N, 4, 1, SMAP><<<grid, dim3(64, 4), lds, s>>>(a);
    }
    return hipGetLastError();
}

template <int N, bool SMAP>
hipError_t launch_pressure_planes(const StepArgs &a, size_t lds, hipStream_t s)
{
    const dim3 grid(8 * a.ptiles_per_xcd);
    if (a.plane_rows == 8) {
        if (a.prs_planes == 8)
            k_pressure_planes<N, 8, 8, SMAP><<<grid, dim3(64, 8), lds, s>>>(a);
        else if (a.prs_planes == 2)
            k_pressure_planes<N, 8, 2, SMAP><<<grid, dim3(64, 8), lds, s>>>(a);
        else
            k_pressure_planes<N, 8, 4, SMAP><<<grid, dim3(64, 8), lds, s>>>(a);
    } else {
        if (a.prs_planes == 8)
            k_pressure_planes<N, 4, 8, SMAP><<<grid, dim3(64, 4), lds, s>>>(a);
        else if (a.prs_planes == 2)
            k_pressure_planes<N, 4, 2, SMAP><<<grid, dim3(64, 4), lds, s>>>(a);
        else
            k_pressure_planes<N, 4, 4, SMAP><<<grid, dim3(64, 4), lds, s>>>(a);
    }
    return hipGetLastError();
}

// 2D tile kernels: 64 x plane_rows tiles (4, 8 or 16 rows), one per block
template <int N, bool SMAP, bool WIDE>
hipError_t launch_tile2d(bool velocity, const StepArgs &a, size_t lds, hipStream_t s)
{
    const dim3 grid(8 * (velocity ? a.vtiles_per_xcd : a.ptiles_per_xcd));
    const dim3 block(64, a.plane_rows);
    if (a.plane_rows == 16) {
        if (velocity)
            k_velocity_tile2d<N, 16, SMAP, WIDE><<<grid, block, lds, s>>>(a);
        else
            k_pressure_tile2d<N, 16, SMAP, WIDE><<<grid, block, lds, s>>>(a);
    } else if (a.plane_rows == 8) {
        if (velocity)
            k_velocity_tile2d<N, 8, SMAP, WIDE><<<grid, block, lds, s>>>(a);
        else
            k_pressure_tile2d<N, 8, SMAP, WIDE><<<grid, block, lds, s>>>(a);
    } else {
        if (velocity)
            k_velocity_tile2d<N, 4, SMAP, WIDE><<<grid, dim3(64, 4), lds, s>>>(a);
        else
            k_pressure_tile2d<N, 4, SMAP, WIDE><<<grid, dim3(64, 4), lds, s>>>(a);
    }
    return hipGetLastError();
}

// 3D launch shapes: (tile rows along y, rows per thread) -> block (64, rows / rpt)
template <int NDIM, int N>
hipError_t launch_nd(bool velocity, int tile_rows, int rpt, const StepArgs &a, hipStream_t s)
{
    if (NDIM != 2 && a.fd_b != 0.0f) return hipErrorNotSupported;
    if constexpr (NDIM == 3) {
        if (velocity && a.plane) {
            const size_t lds = (size_t)a.class_cap * (2 + 2 * N) * sizeof(float);
            return a.amap ? launch_velocity_plane<N, true>(a, lds, s) : launch_velocity_plane<N, false>(a, lds, s);
        }
        if (!velocity && a.plane_p) {
            const size_t lds = (size_t)a.class_cap * (3 + 2 * N) * sizeof(float);
            return a.amap ? launch_pressure_planes<N, true>(a, lds, s) : launch_pressure_planes<N, false>(a, lds, s);
        }
        if (tile_rows == 4) return launch_pair<3, N, 64, 4, 1>(velocity, a, s);
        if (tile_rows == 8 && rpt == 2) return launch_pair<3, N, 64, 4, 2>(velocity, a, s);
        if (tile_rows == 8) return launch_pair<3, N, 64, 8, 1>(velocity, a, s);
        if (rpt == 2) return launch_pair<3, N, 64, 8, 2>(velocity, a, s);
        return launch_pair<3, N, 64, 16, 1>(velocity, a, s);
    } else if constexpr (NDIM == 2) {
        if ((velocity && a.plane) || (!velocity && a.plane_p)) {
            const size_t lds = (size_t)a.class_cap * (velocity ? 2 + 2 * N : 3 + 2 * N) * sizeof(float);
            if (a.fd_b != 0.0f)
                return a.amap ? launch_tile2d<N, true, true>(velocity, a, lds, s)
                              : launch_tile2d<N, false, true>(velocity, a, lds, s);
            return a.amap ? launch_tile2d<N, true, false>(velocity, a, lds, s)
                          : launch_tile2d<N, false, false>(velocity, a, lds, s);
        }
        if (a.fd_b != 0.0f) return hipErrorNotSupported;     // the widened stencil runs on the tile kernels only
        return launch_pair<2, N, 64, 1, 1>(velocity, a, s);
    } else {
        return launch_pair<1, N, 256, 1, 1>(velocity, a, s);
    }
}

template <int NDIM>
hipError_t launch_n(bool velocity, int nmech, int tile_rows, int rpt, const StepArgs &a, hipStream_t s)
{
    switch (nmech) {
    case 1: return launch_nd<NDIM, 1>(velocity, tile_rows, rpt, a, s);
    case 2: return launch_nd<NDIM, 2>(velocity, tile_rows, rpt, a, s);
    case 3: return launch_nd<NDIM, 3>(velocity, tile_rows, rpt, a, s);
    case 4: return launch_nd<NDIM, 4>(velocity, tile_rows, rpt, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_any(bool velocity, int ndim, int nmech, int tile_rows, int rpt, const StepArgs &a, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    switch (ndim) {
    case 1: return launch_n<1>(velocity, nmech, tile_rows, rpt, a, s);
    case 2: return launch_n<2>(velocity, nmech, tile_rows, rpt, a, s);
    case 3: return launch_n<3>(velocity, nmech, tile_rows, rpt, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

void tile_shape(int ndim, int tile_rows, int *tx, int *ty)
{
    if (ndim == 3) {
        *tx = 64;
        *ty = tile_rows;
    } else if (ndim == 2) {
        *tx = 64;
        *ty = 1;
    } else {
        *tx = 256;
        *ty = 1;
    }
}

hipError_t launch_velocity(int ndim, int nmech, int tile_rows, int rpt, const StepArgs &a, hipStream_t s)
{
    return launch_any(true, ndim, nmech, tile_rows, rpt, a, s);
}

hipError_t launch_pressure(int ndim, int nmech, int tile_rows, int rpt, const StepArgs &a, hipStream_t s)
{
    return launch_any(false, ndim, nmech, tile_rows, rpt, a, s);
}

hipError_t launch_src_rec(const SrcRecArgs &a, hipStream_t s)
{
    // one workgroup at least: it advances the step counter
    const int64_t blocks = std::max<int64_t>(1, (a.n_cells + 255) / 256);
    k_src_rec<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace fw
