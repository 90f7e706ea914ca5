// gfx950 kernels of the discrete adjoint of one linear step (beta = 0).
//
// The forward step maps u^n = (p, v, psi1, psi2, psiP1, psiP2) to u^{n+1}.
// Its transpose is applied in reverse order -- pressure sub-step, then
// velocity sub-step -- using div_a = -grad_a^T of the staggered operators
// (summation by parts with zero values beyond the grid).  Besides the adjoint
// state, one reverse step accumulates per cell
//   gK += lam_p^{n+1} * dp^{n+1}/dK   = lam_p^{n+1} * (-dt T^n),
//   gs += sum over the recursions owned by the cell of mu (b_s psi^n + a_s D^n),
// where s scales every d coefficient of the cell (d -> s d) and a_s, b_s are
// the derivatives of Eqs. (relaxation_a)/(relaxation_b) with respect to s.
// Two kernels per reverse step:
//   adj_pressure : lam_p -= sum_a div_a(lamD1_a) of the reverse step before
//                  (the last part of the velocity transpose, which needs the
//                  neighbours' lamD1 and so cannot finish in the kernel that
//                  writes it), then the pointwise transpose of the pressure
//                  update (needs the divergence of the forward v^{n+1/2});
//                  writes lamD2_a.
//   adj_velocity : lam_v -= grad_a(lamD2_a), transpose of the velocity update
//                  (needs grad_a of the forward p^n and the forward CPML
//                  memory variable of u^{n+1}); writes lamD1_a.
// The CPML stage comes first in the forward operators (D_a + psiP_a, then
// the tissue stretch), so its transpose comes last here.
// adj_finish applies the last pending lamD1 after the final reverse step.
// One thread per (x, y) column of a tile, marching the tile's z range (y in
// 2D).  Stencil operands along the marching axis are kept in a register queue
// of eight planes, so each plane of them is read from memory once per tile;
// the in-plane neighbours are direct loads served by the caches.  The memory
// variables use vector accesses.  (Non-temporal hints, which help the step
// kernels, measured about 1 % slower here.)
#include "fw_internal.h"
#include "fw_vec.h"

namespace fw {

namespace {

__device__ __forceinline__ uint64_t splitmix64_a(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float st4(const float (&c)[4], float d1, float d2, float d3, float d4)
{
    return fmaf(c[3], d4, fmaf(c[2], d3, fmaf(c[1], d2, c[0] * d1)));
}

struct Geo {
    int n[3];       // nx, ny, nz
    int st[3];      // strides of x, y, z in the stored layout (rows D.pitch apart)
    int c[3];       // coordinates of the cell
    int g;          // domain-local stored index
    int u;          // domain-local unpadded index (rows nx apart): gradients, speed perturbation
};

// staggered gradient (cell field -> face i+1/2 of axis a), zero beyond the grid
__device__ __forceinline__ float grad_a(const float *__restrict__ f, const Geo &G, int a, const float (&fd)[4])
{
    const int i = G.c[a], n = G.n[a], s = G.st[a], g = G.g;
    float d[4];
#pragma unroll
    for (int m = 1; m <= 4; ++m) {
        const float fp = (i + m < n) ? f[g + m * s] : 0.0f;
        const float fm = (i + 1 - m >= 0) ? f[g + (1 - m) * s] : 0.0f;
        d[m - 1] = fp - fm;
    }
    return st4(fd, d[0], d[1], d[2], d[3]);
}

// staggered divergence term (face field -> cell i of axis a)
__device__ __forceinline__ float div_a(const float *__restrict__ f, const Geo &G, int a, const float (&fd)[4])
{
    const int i = G.c[a], n = G.n[a], s = G.st[a], g = G.g;
    float d[4];
#pragma unroll
    for (int m = 1; m <= 4; ++m) {
        const float fp = (i + m - 1 < n) ? f[g + (m - 1) * s] : 0.0f;
        const float fm = (i - m >= 0) ? f[g - m * s] : 0.0f;
        d[m - 1] = fp - fm;
    }
    return st4(fd, d[0], d[1], d[2], d[3]);
}

template <int NDIM>
__device__ __forceinline__ bool setup(const AdjArgs &A, Tile &T, DomainDesc &D)
{
    const int b = blockIdx.x;
    const int ti = (b & 7) * A.s.tiles_per_xcd + (b >> 3);
    if (ti >= A.s.n_tiles) return false;
    T = A.s.tiles[ti];
    D = A.s.doms[T.dom];
    return true;
}

template <int NDIM>
__device__ __forceinline__ bool column(const Tile &T, const DomainDesc &D, Geo &G)
{
    G.n[0] = (int)D.n[0];
    G.n[1] = (int)D.n[1];
    G.n[2] = (int)D.n[2];
    G.st[0] = 1;
    G.st[1] = D.pitch;
    G.st[2] = D.pitch * G.n[1];
    G.c[0] = T.x0 + (int)threadIdx.x;
    G.c[1] = NDIM == 3 ? T.y0 + (int)threadIdx.y : 0;
    G.c[2] = 0;
    return G.c[0] < G.n[0] && G.c[1] < G.n[1];
}

// march coordinate: z in 3D, y in 2D
template <int NDIM>
__device__ __forceinline__ void at_plane(Geo &G, int z)
{
    if (NDIM == 3) G.c[2] = z;
    if (NDIM == 2) G.c[1] = z;
    G.g = (G.c[2] * G.n[1] + G.c[1]) * G.st[1] + G.c[0];
    G.u = (G.c[2] * G.n[1] + G.c[1]) * G.n[0] + G.c[0];
}

__device__ __forceinline__ bool slab(int c, int n, int P) { return P > 0 && (c < P || c >= n - P); }

// Marching axis (none in 1D, where a tile is one row) and its register queue:
// q[j] holds the operand at marching coordinate first + j, zero beyond the
// grid.  With first = z - 3 the queue serves the gradient of plane z
// (operand at z-3 .. z+4), with first = z - 4 the divergence (z-4 .. z+3);
// both take sum_m c_m (q[3+m] - q[4-m]), the same operations as grad_a and
// div_a.
template <int NDIM>
struct March {
    static constexpr bool on = NDIM >= 2;
    static constexpr int axis = NDIM - 1;
    int col, stride, n;
    __device__ __forceinline__ void init(const Geo &G)
    {
        col = G.c[0] + (NDIM == 3 ? G.c[1] * G.st[1] : 0);
        stride = G.st[axis];
        n = G.n[axis];
    }
    __device__ __forceinline__ float at(const float *__restrict__ f, int zz) const
    {
        return (zz >= 0 && zz < n) ? f[col + zz * stride] : 0.0f;
    }
    __device__ __forceinline__ void fill(float (&q)[8], const float *__restrict__ f, int first) const
    {
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = at(f, first + j);
    }
    __device__ __forceinline__ void push(float (&q)[8], const float *__restrict__ f, int zz) const
    {
#pragma unroll
        for (int j = 0; j < 7; ++j) q[j] = q[j + 1];
        q[7] = zz < n ? f[col + zz * stride] : 0.0f;
    }
};

__device__ __forceinline__ float qdiff(const float (&c)[4], const float (&q)[8])
{
    return st4(c, q[4] - q[3], q[5] - q[2], q[6] - q[1], q[7] - q[0]);
}

template <int NDIM, int N>
__global__ void k_adj_pressure(const AdjArgs A)
{
    Tile T;
    DomainDesc D;
    if (!setup<NDIM>(A, T, D)) return;
    // class tables of the domain in LDS: 1/kappa_2, K, a2, b2, da2/ds, db2/ds
    extern __shared__ float s_tab[];
    const int C = A.s.class_cap;
    float *s_ik = s_tab, *s_K = s_tab + C, *s_a = s_tab + 2 * C, *s_b = s_a + N * C, *s_as = s_b + N * C,
          *s_bs = s_as + N * C;
    {
        const int tid = threadIdx.y * blockDim.x + threadIdx.x, nt = blockDim.x * blockDim.y;
        for (int c = tid; c < D.n_classes; c += nt) {
            const ClassCoef &cc = A.s.classes[D.class_base + c];
            const ClassAdj &ca = A.cadj[D.class_base + c];
            s_ik[c] = cc.ik2;
            s_K[c] = cc.K;
#pragma unroll
            for (int nu = 0; nu < N; ++nu) {
                s_a[nu * C + c] = cc.a2[nu];
                s_b[nu * C + c] = cc.b2[nu];
                s_as[nu * C + c] = ca.a2s[nu];
                s_bs[nu * C + c] = ca.b2s[nu];
            }
        }
    }
    __syncthreads();
    Geo G;
    if (!column<NDIM>(T, D, G)) return;
    const int64_t o = D.cell_off;
    const float dt = A.s.dt;
    const int P = A.s.pml;
    const float *vn[3] = {A.fnext.vx + o, A.fnext.vy + o, A.fnext.vz + o};
    const float *ld1[3] = {A.lamD1[0] + o, A.lamD1[1] + o, A.lamD1[2] + o};
    using MQ = March<NDIM>;
    MQ Q;
    Q.init(G);
    constexpr int ma = MQ::axis;
    float qv[8], ql[8];   // v_ma and lamD1_ma, planes z-4 .. z+3
    if constexpr (MQ::on) {
        Q.fill(qv, vn[ma], T.z0 - 4);
        if (A.fold_div) Q.fill(ql, ld1[ma], T.z0 - 4);
    }
    for (int z = T.z0; z < T.z1; ++z) {
        at_plane<NDIM>(G, z);
        const int g = G.g;
        const int64_t gg = o + g;
        const int L = A.s.f.cls[gg];
        // lam_p^{n+1}: the pending divergence of the velocity transpose
        float lp = A.lam.p[gg];
        if (A.fold_div) {
            float acc = 0.0f;
#pragma unroll
            for (int a = 0; a < NDIM; ++a) {
                if (MQ::on && a == ma)
                    acc += qdiff(A.s.fd, ql);
                else
                    acc += div_a(ld1[a], G, a, A.s.fd);
            }
            lp -= acc;
            A.lam.p[gg] = lp;
            if constexpr (MQ::on) Q.push(ql, ld1[ma], z + 4);
        }
        // forward divergence of v^{n+1/2} (state u^{n+1}) after the CPML
        // stage: D_a + psiP2_a^{n+1} in the slab of axis a
        float Dd[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int a = 0; a < NDIM; ++a) {
            if (MQ::on && a == ma)
                Dd[a] = qdiff(A.s.fd, qv);
            else
                Dd[a] = div_a(vn[a], G, a, A.s.fd);
            if (slab(G.c[a], G.n[a], P)) Dd[a] += A.fnext.pP2[a][gg];
        }
        if constexpr (MQ::on) Q.push(qv, vn[ma], z + 4);
        float S = Dd[0];
#pragma unroll
        for (int a = 1; a < NDIM; ++a) S += Dd[a];
        // T^n from the updated memory variables of u^{n+1}
        float psn[N], psf[N], lps[N];
        load_vec<N>(A.fnext.psi2 + gg * N, psn);
        load_vec<N>(A.s.f.psi2 + gg * N, psf);
        load_vec<N>(A.lam.psi2 + gg * N, lps);
        float Tt = s_ik[L] * S;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) Tt += psn[nu];
        float K = s_K[L];
        if (A.s.noise_amp != 0.0f) {
            const uint64_t h = splitmix64_a(D.noise_seed ^ (uint64_t)(uint32_t)G.u);
            const float u = (float)(h >> 40) * 0x1.0p-24f;
            const float e = A.s.noise_amp * fmaf(2.0f, u, -1.0f);
            const float f1 = 1.0f + e;
            K = K * (f1 * f1);
        }
        const int64_t pk = D.packed_off + G.u;
        const float gk0 = A.gK[pk];
        A.gK[pk] = gk0 + lp * (-dt * Tt);
        const float q = -dt * K * lp;
        float gdiv = s_ik[L] * q;
        float gsum = 0.0f;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            const float mu = lps[nu] + q;
            gdiv = fmaf(s_a[nu * C + L], mu, gdiv);
            gsum = fmaf(mu, fmaf(s_as[nu * C + L], S, s_bs[nu * C + L] * psf[nu]), gsum);
            lps[nu] = s_b[nu * C + L] * mu;
        }
        store_vec<N>(A.lam.psi2 + gg * N, lps);
        // gdiv is the adjoint of the CPML-stretched divergence of each axis;
        // transpose of D_a + psiP2_a, psiP2_a <- bC psiP2_a + aC D_a
#pragma unroll
        for (int a = 0; a < NDIM; ++a) {
            float ld = gdiv;
            if (slab(G.c[a], G.n[a], P)) {
                const int32_t off = D.pml_off[a];
                const float aC = A.s.pml_tab[off + 2 * G.n[a] + G.c[a]];
                const float bC = A.s.pml_tab[off + 3 * G.n[a] + G.c[a]];
                const float mu = A.lam.pP2[a][gg] + gdiv;
                ld = fmaf(aC, mu, gdiv);
                A.lam.pP2[a][gg] = bC * mu;
            }
            A.lamD2[a][gg] = ld;
        }
        const float gs0 = A.gs[pk];
        A.gs[pk] = gs0 + gsum;
    }
}

template <int NDIM, int N>
__global__ void k_adj_velocity(const AdjArgs A)
{
    Tile T;
    DomainDesc D;
    if (!setup<NDIM>(A, T, D)) return;
    // class tables of the domain in LDS: 1/kappa_1, rho, a1, b1, da1/ds, db1/ds
    extern __shared__ float s_tab[];
    const int C = A.s.class_cap;
    float *s_ik = s_tab, *s_rho = s_tab + C, *s_a = s_tab + 2 * C, *s_b = s_a + N * C, *s_as = s_b + N * C,
          *s_bs = s_as + N * C;
    {
        const int tid = threadIdx.y * blockDim.x + threadIdx.x, nt = blockDim.x * blockDim.y;
        for (int c = tid; c < D.n_classes; c += nt) {
            const ClassCoef &cc = A.s.classes[D.class_base + c];
            const ClassAdj &ca = A.cadj[D.class_base + c];
            s_ik[c] = cc.ik1;
            s_rho[c] = cc.rho;
#pragma unroll
            for (int nu = 0; nu < N; ++nu) {
                s_a[nu * C + c] = cc.a1[nu];
                s_b[nu * C + c] = cc.b1[nu];
                s_as[nu * C + c] = ca.a1s[nu];
                s_bs[nu * C + c] = ca.b1s[nu];
            }
        }
    }
    __syncthreads();
    Geo G;
    if (!column<NDIM>(T, D, G)) return;
    const int64_t o = D.cell_off;
    const float dt = A.s.dt;
    const int P = A.s.pml;
    float *lvx[3] = {A.lam.vx, A.lam.vy, A.lam.vz};
    const float *psi1f[3] = {A.s.f.psi1x, A.s.f.psi1y, A.s.f.psi1z};
    float *psi1l[3] = {A.lam.psi1x, A.lam.psi1y, A.lam.psi1z};
    const float *pP1n[3] = {A.fnext.pP1[0], A.fnext.pP1[1], A.fnext.pP1[2]};
    using MQ = March<NDIM>;
    MQ Q;
    Q.init(G);
    constexpr int ma = MQ::axis;
    const float *pf0 = A.s.f.p + o;
    const float *ld2m = A.lamD2[ma] + o;
    float qp[8], ql[8];   // p and lamD2_ma, planes z-3 .. z+4
    if constexpr (MQ::on) {
        Q.fill(qp, pf0, T.z0 - 3);
        Q.fill(ql, ld2m, T.z0 - 3);
    }
    for (int z = T.z0; z < T.z1; ++z) {
        at_plane<NDIM>(G, z);
        const int g = G.g;
        const int64_t gg = o + g;
        const int L = A.s.f.cls[gg];
        float gsum = 0.0f;
#pragma unroll
        for (int a = 0; a < NDIM; ++a) {
            const int i = G.c[a];
            const int Ln = (i + 1 < G.n[a]) ? A.s.f.cls[gg + G.st[a]] : L;
            const float m = 2.0f * dt / (s_rho[L] + s_rho[Ln]);
            const bool mq = MQ::on && a == ma;
            const float lv = lvx[a][gg] - (mq ? qdiff(A.s.fd, ql) : grad_a(A.lamD2[a] + o, G, a, A.s.fd));
            const float r = -m * lv;
            // forward gradient of p^n after the CPML stage
            float D1 = mq ? qdiff(A.s.fd, qp) : grad_a(pf0, G, a, A.s.fd);
            const bool sl = slab(i, G.n[a], P);
            if (sl) D1 += pP1n[a][gg];
            float pf[N], pl[N];
            load_vec<N>(psi1f[a] + gg * N, pf);
            load_vec<N>(psi1l[a] + gg * N, pl);
            float ld = s_ik[L] * r;
#pragma unroll
            for (int nu = 0; nu < N; ++nu) {
                const float mu = pl[nu] + r;
                ld = fmaf(s_a[nu * C + L], mu, ld);
                gsum = fmaf(mu, fmaf(s_as[nu * C + L], D1, s_bs[nu * C + L] * pf[nu]), gsum);
                pl[nu] = s_b[nu * C + L] * mu;
            }
            store_vec<N>(psi1l[a] + gg * N, pl);
            // ld is the adjoint of the CPML-stretched gradient; transpose of
            // D + psiP1, psiP1 <- bF psiP1 + aF D
            if (sl) {
                const int32_t off = D.pml_off[a];
                const float aF = A.s.pml_tab[off + i];
                const float bF = A.s.pml_tab[off + G.n[a] + i];
                const float mu = A.lam.pP1[a][gg] + ld;
                ld = fmaf(aF, mu, ld);
                A.lam.pP1[a][gg] = bF * mu;
            }
            lvx[a][gg] = lv;
            A.lamD1[a][gg] = ld;
        }
        if constexpr (MQ::on) {
            Q.push(qp, pf0, z + 5);
            Q.push(ql, ld2m, z + 5);
        }
        const int64_t pk = D.packed_off + G.u;
        const float gs0 = A.gs[pk];
        A.gs[pk] = gs0 + gsum;
    }
}

template <int NDIM>
__global__ void k_adj_finish(const AdjArgs A)
{
    Tile T;
    DomainDesc D;
    if (!setup<NDIM>(A, T, D)) return;
    Geo G;
    if (!column<NDIM>(T, D, G)) return;
    const int64_t o = D.cell_off;
    for (int z = T.z0; z < T.z1; ++z) {
        at_plane<NDIM>(G, z);
        float acc = 0.0f;
#pragma unroll
        for (int a = 0; a < NDIM; ++a) acc += div_a(A.lamD1[a] + o, G, a, A.s.fd);
        A.lam.p[o + G.g] -= acc;
    }
}

// lam_p[cell] += sum of the residuals of the receivers at that cell; one
// thread per distinct receiver cell, fixed summation order.
__global__ __launch_bounds__(1024) void k_adj_inject(const AdjInjectArgs A)
{
    const int64_t t = A.step;
    for (int64_t u = threadIdx.x; u < A.n_cells; u += blockDim.x) {
        float s = 0.0f;
        for (int32_t k = A.offsets[u]; k < A.offsets[u + 1]; ++k) s += A.res[t * A.n_rec + A.rec_index[k]];
        A.lam_p[A.cells[u]] += s;
    }
}

template <int NDIM, int N>
hipError_t adj_launch(int which, const AdjArgs &a, hipStream_t s)
{
    int tx, ty;
    tile_shape(NDIM, a.tile_rows, &tx, &ty);
    const dim3 block(tx, NDIM == 3 ? ty : 1);
    const dim3 grid(8 * a.s.tiles_per_xcd);
    const size_t lds = (size_t)a.s.class_cap * (2 + 4 * N) * sizeof(float);
    if (which == 0)
        k_adj_pressure<NDIM, N><<<grid, block, lds, s>>>(a);
    else if (which == 1)
        k_adj_velocity<NDIM, N><<<grid, block, lds, s>>>(a);
    else
        k_adj_finish<NDIM><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

// dJ/dc and dJ/dalpha0 per cell (one thread per cell of the unpadded
// layout).  The speed perturbation is evaluated exactly as in the forward
// pressure update (same hash, same FP32 operations), so (1 + eps)^2 matches
// the factor the modulus of the run was built with.
__global__ __launch_bounds__(256) void k_adj_chain(const AdjChainArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.n_packed) return;
    int lo = 0, hi = A.n_domains - 1;   // domain holding unpadded cell i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.doms[mid].packed_off <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    const DomainDesc &D = A.doms[lo];
    const int64_t g = i - D.packed_off;                       // unpadded local index
    const int64_t nx = D.n[0];
    const int64_t stored = (g / nx) * D.pitch + g % nx;       // its place in the padded rows
    const float2 ch = A.chain[D.class_base + A.cls[D.cell_off + stored]];
    float f2 = 1.0f;
    if (A.noise_amp != 0.0f) {
        const uint64_t h = splitmix64_a(D.noise_seed ^ (uint64_t)(uint32_t)g);
        const float u = (float)(h >> 40) * 0x1.0p-24f;
        const float e = A.noise_amp * fmaf(2.0f, u, -1.0f);
        const float f1 = 1.0f + e;
        f2 = f1 * f1;
    }
    A.grad_c[i] = fmaf(ch.x * f2, A.gK[i], A.grad_c[i]);
    if (A.grad_a0) A.grad_a0[i] = fmaf(A.gs[i], ch.y, A.grad_a0[i]);
}

template <int NDIM>
hipError_t adj_launch_n(int which, int nmech, const AdjArgs &a, hipStream_t s)
{
    switch (nmech) {
    case 1: return adj_launch<NDIM, 1>(which, a, s);
    case 2: return adj_launch<NDIM, 2>(which, a, s);
    case 3: return adj_launch<NDIM, 3>(which, a, s);
    case 4: return adj_launch<NDIM, 4>(which, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t adj_launch_dim(int which, int ndim, int nmech, const AdjArgs &a, hipStream_t s)
{
    if (ndim == 1) return adj_launch_n<1>(which, nmech, a, s);
    if (ndim == 2) return adj_launch_n<2>(which, nmech, a, s);
    if (ndim == 3) return adj_launch_n<3>(which, nmech, a, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_adjoint_step(int ndim, int nmech, const AdjArgs &a, hipStream_t s)
{
    if (a.s.n_tiles <= 0) return hipSuccess;
    hipError_t e = adj_launch_dim(0, ndim, nmech, a, s);
    if (e != hipSuccess) return e;
    return adj_launch_dim(1, ndim, nmech, a, s);
}

hipError_t launch_adjoint_finish(int ndim, const AdjArgs &a, hipStream_t s)
{
    if (a.s.n_tiles <= 0) return hipSuccess;
    return adj_launch_dim(2, ndim, 1, a, s);
}

hipError_t launch_adjoint_chain(const AdjChainArgs &a, hipStream_t s)
{
    if (a.n_packed <= 0) return hipSuccess;
    const int64_t blocks = (a.n_packed + 255) / 256;
    if (blocks > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    k_adj_chain<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_adjoint_inject(const AdjInjectArgs &a, hipStream_t s)
{
    if (a.n_cells <= 0) return hipSuccess;
    k_adj_inject<<<dim3(1), dim3(1024), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace fw
