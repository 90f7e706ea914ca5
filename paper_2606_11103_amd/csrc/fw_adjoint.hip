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
// 2D grids with the tile kernels on (the default) run the two reverse-step
// kernels on 64 x R tiles with LDS halos (k_adj_*_tile2d); otherwise one
// thread per (x, y) column of a tile marches the tile's z range (y in 2D).  Stencil operands along the marching axis are kept in a register queue
// of eight planes, so each plane of them is read from memory once per tile;
// the in-plane neighbours are direct loads served by the caches.  The memory
// variables use vector accesses.  (Non-temporal hints, which help the step
// kernels, measured about 1 % slower here.)
#include "fw_internal.h"
#include "fw_vec.h"

namespace fw {

namespace {


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
    return stencil4(fd, d[0], d[1], d[2], d[3]);
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
    return stencil4(fd, d[0], d[1], d[2], d[3]);
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
    return stencil4(c, q[4] - q[3], q[5] - q[2], q[6] - q[1], q[7] - q[0]);
}

// Pointwise parts of the two transposes at one cell, shared by the marching
// and the 2D tile kernels so that both give the same bits.  Each is split
// into the loads of the cell's own operands (a struct the tile kernels fill
// before their LDS barrier, so those loads overlap the halo staging) and the
// arithmetic on them.
// EARLY: the gradient sums and the adjoint CPML variables are loaded with the
// rest (tile kernels); otherwise where they are used (the marching kernels,
// whose register queues leave less room for operands held early).
// own-cell accesses: plain (marching kernels: non-temporal hints measured
// about 1 % slower there), or non-temporal (NT, tile kernels: the caches then
// keep the halo rows that neighbouring tiles read again; 439 / 343 us against
// 465 / 375 us per reverse step of 16 x 1024^2 at N = 4)
template <int N, bool NT>
__device__ __forceinline__ void ldv(const float *__restrict__ p, float (&v)[N])
{
    if constexpr (NT)
        load_stream<N>(p, v);
    else
        load_vec<N>(p, v);
}
template <int N, bool NT>
__device__ __forceinline__ void stv(float *__restrict__ p, const float (&v)[N])
{
    if constexpr (NT)
        store_stream<N>(p, v);
    else
        store_vec<N>(p, v);
}
template <bool NT>
__device__ __forceinline__ float ld1(const float *__restrict__ p)
{
    if constexpr (NT)
        return load1_stream(p);
    else
        return *p;
}
template <bool NT>
__device__ __forceinline__ void st1(float *__restrict__ p, float v)
{
    if constexpr (NT)
        store1_stream(p, v);
    else
        *p = v;
}

template <int NDIM, int N, bool EARLY>
struct AdjPressureIn {
    float psn[N], psf[N], lps[N];   // psi2 of u^{n+1}, of u^n, and its adjoint
    float gk0, gs0, lpp[NDIM];      // gradient sums so far; adjoint CPML variables (slab cells)
};

template <int NDIM, int N, bool EARLY, bool NT = false>
__device__ __forceinline__ void adj_pressure_load(const AdjArgs &A, const DomainDesc &D, int64_t gg, int u,
                                                  const int (&c)[3], const int (&n)[3],
                                                  AdjPressureIn<NDIM, N, EARLY> &o)
{
    ldv<N, NT>(A.fnext.psi2 + gg * N, o.psn);
    ldv<N, NT>(A.s.f.psi2 + gg * N, o.psf);
    ldv<N, NT>(A.lam.psi2 + gg * N, o.lps);
    if constexpr (EARLY) {
        const int64_t pk = D.packed_off + u;
        o.gk0 = ld1<NT>(A.gK + pk);
        o.gs0 = ld1<NT>(A.gs + pk);
#pragma unroll
        for (int a = 0; a < NDIM; ++a) o.lpp[a] = slab(c[a], n[a], A.s.pml) ? A.lam.pP2[a][gg] : 0.0f;
    }
}

// lp is lam_p^{n+1} with the pending divergence applied, S the forward
// divergence of v^{n+1/2} after the CPML stage; LDS class tables as in
// k_adj_pressure.
template <int NDIM, int N, bool EARLY, bool NT = false>
__device__ __forceinline__ void adj_pressure_cell(const AdjArgs &A, const DomainDesc &D, const float *s_tab,
                                                  int C, int64_t gg, int u, const int (&c)[3], const int (&n)[3],
                                                  int L, float lp, float S, AdjPressureIn<NDIM, N, EARLY> &o)
{
    const float *s_ik = s_tab, *s_K = s_tab + C, *s_a = s_tab + 2 * C, *s_b = s_a + N * C, *s_as = s_b + N * C,
                *s_bs = s_as + N * C;
    const float dt = A.s.dt;
    const int P = A.s.pml;
    // T^n from the updated memory variables of u^{n+1}
    float Tt = s_ik[L] * S;
#pragma unroll
    for (int nu = 0; nu < N; ++nu) Tt += o.psn[nu];
    float K = s_K[L];
    if (A.s.noise_amp != 0.0f) K = K * speed_factor_sq(D.noise_seed, (uint32_t)u, A.s.noise_amp);
    const int64_t pk = D.packed_off + u;
    const float gk0 = EARLY ? o.gk0 : A.gK[pk];
    st1<NT>(A.gK + pk, gk0 + lp * (-dt * Tt));
    const float q = -dt * K * lp;
    float gdiv = s_ik[L] * q;
    float gsum = 0.0f;
#pragma unroll
    for (int nu = 0; nu < N; ++nu) {
        const float mu = o.lps[nu] + q;
        gdiv = fmaf(s_a[nu * C + L], mu, gdiv);
        gsum = fmaf(mu, fmaf(s_as[nu * C + L], S, s_bs[nu * C + L] * o.psf[nu]), gsum);
        o.lps[nu] = s_b[nu * C + L] * mu;
    }
    stv<N, NT>(A.lam.psi2 + gg * N, o.lps);
    // gdiv is the adjoint of the CPML-stretched divergence of each axis;
    // transpose of D_a + psiP2_a, psiP2_a <- bC psiP2_a + aC D_a
#pragma unroll
    for (int a = 0; a < NDIM; ++a) {
        float ld = gdiv;
        if (slab(c[a], n[a], P)) {
            const int32_t off = D.pml_off[a];
            const float aC = A.s.pml_tab[off + 2 * n[a] + c[a]];
            const float bC = A.s.pml_tab[off + 3 * n[a] + c[a]];
            const float mu = (EARLY ? o.lpp[a] : A.lam.pP2[a][gg]) + gdiv;
            ld = fmaf(aC, mu, gdiv);
            A.lam.pP2[a][gg] = bC * mu;
        }
        A.lamD2[a][gg] = ld;
    }
    const float gs0 = EARLY ? o.gs0 : A.gs[pk];
    st1<NT>(A.gs + pk, gs0 + gsum);
}

template <int N>
struct AdjVelocityIn {
    float lv0;                      // lam_v of the axis before this step
    float pf[N], pl[N];             // psi1 of u^n and its adjoint
};

template <int N, bool NT = false>
__device__ __forceinline__ void adj_velocity_load(const AdjArgs &A, int a, int64_t gg, AdjVelocityIn<N> &o)
{
    const float *lvx = a == 0 ? A.lam.vx : (a == 1 ? A.lam.vy : A.lam.vz);
    const float *psi1f = a == 0 ? A.s.f.psi1x : (a == 1 ? A.s.f.psi1y : A.s.f.psi1z);
    const float *psi1l = a == 0 ? A.lam.psi1x : (a == 1 ? A.lam.psi1y : A.lam.psi1z);
    o.lv0 = ld1<NT>(lvx + gg);
    ldv<N, NT>(psi1f + gg * N, o.pf);
    ldv<N, NT>(psi1l + gg * N, o.pl);
}

// Axis a: lv = lam_v after the gradient of lamD2, r = -m lv, D1 the forward
// gradient of p^n before the CPML stage.  Accumulates the cell's d-scale
// term into gsum.
template <int N, bool NT = false>
__device__ __forceinline__ void adj_velocity_axis(const AdjArgs &A, const DomainDesc &D, const float *s_tab, int C,
                                                  int a, int i, int n, int64_t gg, int L, float lv, float r,
                                                  float D1, AdjVelocityIn<N> &o, float &gsum)
{
    const float *s_ik = s_tab, *s_a = s_tab + 2 * C, *s_b = s_a + N * C, *s_as = s_b + N * C, *s_bs = s_as + N * C;
    float *lvx = a == 0 ? A.lam.vx : (a == 1 ? A.lam.vy : A.lam.vz);
    float *psi1l = a == 0 ? A.lam.psi1x : (a == 1 ? A.lam.psi1y : A.lam.psi1z);
    // forward gradient of p^n after the CPML stage
    const bool sl = slab(i, n, A.s.pml);
    if (sl) D1 += A.fnext.pP1[a][gg];
    float ld = s_ik[L] * r;
#pragma unroll
    for (int nu = 0; nu < N; ++nu) {
        const float mu = o.pl[nu] + r;
        ld = fmaf(s_a[nu * C + L], mu, ld);
        gsum = fmaf(mu, fmaf(s_as[nu * C + L], D1, s_bs[nu * C + L] * o.pf[nu]), gsum);
        o.pl[nu] = s_b[nu * C + L] * mu;
    }
    stv<N, NT>(psi1l + gg * N, o.pl);
    // ld is the adjoint of the CPML-stretched gradient; transpose of
    // D + psiP1, psiP1 <- bF psiP1 + aF D
    if (sl) {
        const int32_t off = D.pml_off[a];
        const float aF = A.s.pml_tab[off + i];
        const float bF = A.s.pml_tab[off + n + i];
        const float mu = A.lam.pP1[a][gg] + ld;
        ld = fmaf(aF, mu, ld);
        A.lam.pP1[a][gg] = bF * mu;
    }
    st1<NT>(lvx + gg, lv);
    A.lamD1[a][gg] = ld;
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
        AdjPressureIn<NDIM, N, false> in;
        adj_pressure_load<NDIM, N, false>(A, D, gg, G.u, G.c, G.n, in);
        adj_pressure_cell<NDIM, N, false>(A, D, s_tab, C, gg, G.u, G.c, G.n, L, lp, S, in);
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
            const float gl = mq ? qdiff(A.s.fd, ql) : grad_a(A.lamD2[a] + o, G, a, A.s.fd);
            const float D1 = mq ? qdiff(A.s.fd, qp) : grad_a(pf0, G, a, A.s.fd);
            AdjVelocityIn<N> in;
            adj_velocity_load<N>(A, a, gg, in);
            const float lv = in.lv0 - gl;
            const float r = -m * lv;
            adj_velocity_axis<N>(A, D, s_tab, C, a, i, G.n[a], gg, L, lv, r, D1, in, gsum);
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

// 2D tile forms of the two reverse-step kernels: one 64 x TY tile per block
// (the forward tile kernels' list), every stencil operand staged once in LDS
// with a 4-cell halo on each side (zero beyond the grid) instead of the
// marching queue and the direct x-neighbour loads.  A thread keeps only its
// own cell, so more waves fit on a SIMD and each operand is fetched once per
// tile plus its halo; the cell's own operands use non-temporal accesses.  The
// per-cell arithmetic is the marching kernels' own (adj_pressure_cell,
// adj_velocity_axis) with the stencil sums in the same order, so the results
// are identical.
template <int TY>
struct AdjTile2 {
    static constexpr int BX = 64, LX = BX + 8, LY = TY + 8, NT = BX * TY;
    static constexpr int YSL = (8 * BX + NT - 1) / NT;   // y-halo slots per thread
};

// LDS image of field f over the tile's rows, columns x0 - 4 .. x0 + 67
// (TY x LX, own value written by the caller): x-halo slot of thread tid
template <int TY>
__device__ __forceinline__ void stage_xhalo(float *dst, const float *__restrict__ f, const Tile &T, int nx, int ny,
                                            int px, int tid, int row_off)
{
    using K = AdjTile2<TY>;
    if (tid < 8 * TY) {
        const int row = tid >> 3, k = tid & 7, hx = k < 4 ? k : K::BX + k;
        const int gx = T.x0 - 4 + hx, gy = T.y0 + row;
        dst[(row + row_off) * K::LX + hx] = (gx >= 0 && gx < nx && gy < ny) ? f[gy * px + gx] : 0.0f;
    }
}

// LDS image of field f over the tile's columns, rows y0 - 4 .. y0 + TY + 3
// ((TY + 8) x pitch lx, columns from col_off): y-halo slots of thread tid
template <int TY>
__device__ __forceinline__ void stage_yhalo(float *dst, const float *__restrict__ f, const Tile &T, int nx, int ny,
                                            int px, int tid, int lx, int col_off)
{
    using K = AdjTile2<TY>;
#pragma unroll
    for (int s = 0; s < K::YSL; ++s) {
        const int h = tid + s * K::NT;
        if (h < 8 * K::BX) {
            const int rr = h >> 6, hx = h & 63, hy = rr < 4 ? rr : TY + rr;
            const int gx = T.x0 + hx, gy = T.y0 - 4 + hy;
            dst[hy * lx + hx + col_off] = (gx < nx && gy >= 0 && gy < ny) ? f[gy * px + gx] : 0.0f;
        }
    }
}

template <int N, int TY>
__global__ __launch_bounds__(64 * TY) void k_adj_pressure_tile2d(const AdjArgs A)
{
    using K = AdjTile2<TY>;
    constexpr int BX = K::BX, LX = K::LX, LY = K::LY;
    __shared__ float s_v0[TY * LX], s_l0[TY * LX];   // v_x, lamD1_x: tile rows, x-halo of 4
    __shared__ float s_v1[LY * BX], s_l1[LY * BX];   // v_y, lamD1_y: tile columns, y-halo of 4
    extern __shared__ float s_tab[];
    const int C = A.s.class_cap;
    const int b = blockIdx.x;
    const int ti = (b & 7) * A.s.vtiles_per_xcd + (b >> 3);
    if (ti >= A.s.n_vtiles) return;
    const Tile T = A.s.vtiles[ti];
    if (T.z1 <= T.z0) return;      // padding of the banded list
    const DomainDesc D = A.s.doms[T.dom];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    {
        float *s_ik = s_tab, *s_K = s_tab + C, *s_a = s_tab + 2 * C, *s_b = s_a + N * C, *s_as = s_b + N * C,
              *s_bs = s_as + N * C;
        for (int c = tid; c < D.n_classes; c += K::NT) {
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
    const int nx = (int)D.n[0], ny = (int)D.n[1], px = D.pitch;
    const int x = T.x0 + tx, y = T.y0 + ty;
    const bool ok = x < nx && y < ny;
    const int64_t o = D.cell_off;
    const int g = y * px + x;
    const int64_t gg = o + g;
    const float *vn0 = A.fnext.vx + o, *vn1 = A.fnext.vy + o;
    const float *lq0 = A.lamD1[0] + o, *lq1 = A.lamD1[1] + o;
    const bool fold = A.fold_div != 0;
    s_v0[ty * LX + 4 + tx] = ok ? vn0[g] : 0.0f;
    s_v1[(ty + 4) * BX + tx] = ok ? vn1[g] : 0.0f;
    stage_xhalo<TY>(s_v0, vn0, T, nx, ny, px, tid, 0);
    stage_yhalo<TY>(s_v1, vn1, T, nx, ny, px, tid, BX, 0);
    if (fold) {
        s_l0[ty * LX + 4 + tx] = ok ? lq0[g] : 0.0f;
        s_l1[(ty + 4) * BX + tx] = ok ? lq1[g] : 0.0f;
        stage_xhalo<TY>(s_l0, lq0, T, nx, ny, px, tid, 0);
        stage_yhalo<TY>(s_l1, lq1, T, nx, ny, px, tid, BX, 0);
    }
    // the cell's own operands, in flight with the staging loads
    const int P = A.s.pml;
    const int c[3] = {x, y, 0}, n[3] = {nx, ny, 1};
    int L = 0;
    float lp = 0.0f, pq[2] = {0.0f, 0.0f};
    constexpr bool NT = true;
    AdjPressureIn<2, N, true> in;
    if (ok) {
        L = A.s.f.cls[gg];
        lp = ld1<NT>(A.lam.p + gg);
        if (slab(x, nx, P)) pq[0] = A.fnext.pP2[0][gg];
        if (slab(y, ny, P)) pq[1] = A.fnext.pP2[1][gg];
        adj_pressure_load<2, N, true, NT>(A, D, gg, y * nx + x, c, n, in);
    }
    __syncthreads();
    if (!ok) return;
    // lam_p^{n+1}: the pending divergence of the velocity transpose
    if (fold) {
        const float *l0 = s_l0 + ty * LX + 4 + tx, *l1 = s_l1 + (ty + 4) * BX + tx;
        float acc = 0.0f;
        acc += stencil4(A.s.fd, l0[0] - l0[-1], l0[1] - l0[-2], l0[2] - l0[-3], l0[3] - l0[-4]);
        acc += stencil4(A.s.fd, l1[0] - l1[-BX], l1[BX] - l1[-2 * BX], l1[2 * BX] - l1[-3 * BX], l1[3 * BX] - l1[-4 * BX]);
        lp -= acc;
        st1<NT>(A.lam.p + gg, lp);
    }
    // forward divergence of v^{n+1/2} (state u^{n+1}) after the CPML stage
    const float *v0 = s_v0 + ty * LX + 4 + tx, *v1 = s_v1 + (ty + 4) * BX + tx;
    float Dd[2];
    Dd[0] = stencil4(A.s.fd, v0[0] - v0[-1], v0[1] - v0[-2], v0[2] - v0[-3], v0[3] - v0[-4]);
    if (slab(x, nx, P)) Dd[0] += pq[0];
    Dd[1] = stencil4(A.s.fd, v1[0] - v1[-BX], v1[BX] - v1[-2 * BX], v1[2 * BX] - v1[-3 * BX], v1[3 * BX] - v1[-4 * BX]);
    if (slab(y, ny, P)) Dd[1] += pq[1];
    float S = Dd[0];
    S += Dd[1];
    adj_pressure_cell<2, N, true, NT>(A, D, s_tab, C, gg, y * nx + x, c, n, L, lp, S, in);
}

template <int N, int TY>
__global__ __launch_bounds__(64 * TY) void k_adj_velocity_tile2d(const AdjArgs A)
{
    using K = AdjTile2<TY>;
    constexpr int BX = K::BX, LX = K::LX, LY = K::LY, CX = BX + 1;
    __shared__ float s_p[LY * LX];                   // p: tile with x- and y-halos of 4
    __shared__ float s_l0[TY * LX];                  // lamD2_x: tile rows, x-halo of 4
    __shared__ float s_l1[LY * BX];                  // lamD2_y: tile columns, y-halo of 4
    __shared__ uint8_t s_c[(TY + 1) * CX];           // classes, plus column x0 + 64 and row y0 + TY
    extern __shared__ float s_tab[];
    const int C = A.s.class_cap;
    const int b = blockIdx.x;
    const int ti = (b & 7) * A.s.vtiles_per_xcd + (b >> 3);
    if (ti >= A.s.n_vtiles) return;
    const Tile T = A.s.vtiles[ti];
    if (T.z1 <= T.z0) return;      // padding of the banded list
    const DomainDesc D = A.s.doms[T.dom];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    {
        float *s_ik = s_tab, *s_rho = s_tab + C, *s_a = s_tab + 2 * C, *s_b = s_a + N * C, *s_as = s_b + N * C,
              *s_bs = s_as + N * C;
        for (int c = tid; c < D.n_classes; c += K::NT) {
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
    const int nx = (int)D.n[0], ny = (int)D.n[1], px = D.pitch;
    const int x = T.x0 + tx, y = T.y0 + ty;
    const bool ok = x < nx && y < ny;
    const int64_t o = D.cell_off;
    const int g = y * px + x;
    const int64_t gg = o + g;
    const float *pf0 = A.s.f.p + o, *l20 = A.lamD2[0] + o, *l21 = A.lamD2[1] + o;
    const uint8_t *cls = A.s.f.cls + o;
    s_p[(ty + 4) * LX + 4 + tx] = ok ? pf0[g] : 0.0f;
    stage_xhalo<TY>(s_p, pf0, T, nx, ny, px, tid, 4);
    stage_yhalo<TY>(s_p, pf0, T, nx, ny, px, tid, LX, 4);
    s_l0[ty * LX + 4 + tx] = ok ? l20[g] : 0.0f;
    stage_xhalo<TY>(s_l0, l20, T, nx, ny, px, tid, 0);
    s_l1[(ty + 4) * BX + tx] = ok ? l21[g] : 0.0f;
    stage_yhalo<TY>(s_l1, l21, T, nx, ny, px, tid, BX, 0);
    const int L0 = ok ? (int)cls[g] : 0;
    s_c[ty * CX + tx] = (uint8_t)L0;
    if (tid < TY + BX) {
        int gx, gy, li;
        if (tid < TY) {
            gx = T.x0 + BX;
            gy = T.y0 + tid;
            li = tid * CX + BX;
        } else {
            gx = T.x0 + (tid - TY);
            gy = T.y0 + TY;
            li = TY * CX + (tid - TY);
        }
        s_c[li] = (gx < nx && gy < ny) ? cls[gy * px + gx] : (uint8_t)0;
    }
    // the cell's own operands of each axis are loaded after the barrier, right
    // before their use (issuing them with the staging loads needs more
    // registers: 488 against 465 us per reverse step of 16 x 1024^2, N = 4)
    constexpr bool NT = true;
    AdjVelocityIn<N> in0, in1;
    float gs0 = 0.0f;
    const int64_t pk = D.packed_off + (int64_t)y * nx + x;
    if (ok) gs0 = ld1<NT>(A.gs + pk);
    __syncthreads();
    if (!ok) return;
    adj_velocity_load<N, NT>(A, 0, gg, in0);
    const float *s_rho = s_tab + C;
    const float dt = A.s.dt;
    const int L = L0;
    const float *sp = s_p + (ty + 4) * LX + 4 + tx;
    const float *l0 = s_l0 + ty * LX + 4 + tx, *l1 = s_l1 + (ty + 4) * BX + tx;
    float gsum = 0.0f;
    {   // x: gradient over the row, lamD2_x and p at x - 3 .. x + 4
        const int Ln = (x + 1 < nx) ? s_c[ty * CX + tx + 1] : L;
        const float m = 2.0f * dt / (s_rho[L] + s_rho[Ln]);
        const float lv = in0.lv0 - stencil4(A.s.fd, l0[1] - l0[0], l0[2] - l0[-1], l0[3] - l0[-2], l0[4] - l0[-3]);
        const float r = -m * lv;
        const float D1 = stencil4(A.s.fd, sp[1] - sp[0], sp[2] - sp[-1], sp[3] - sp[-2], sp[4] - sp[-3]);
        adj_velocity_axis<N, NT>(A, D, s_tab, C, 0, x, nx, gg, L, lv, r, D1, in0, gsum);
    }
    adj_velocity_load<N, NT>(A, 1, gg, in1);
    {   // y: gradient over the column
        const int Ln = (y + 1 < ny) ? s_c[(ty + 1) * CX + tx] : L;
        const float m = 2.0f * dt / (s_rho[L] + s_rho[Ln]);
        const float lv = in1.lv0 - stencil4(A.s.fd, l1[BX] - l1[0], l1[2 * BX] - l1[-BX], l1[3 * BX] - l1[-2 * BX],
                                       l1[4 * BX] - l1[-3 * BX]);
        const float r = -m * lv;
        const float D1 = stencil4(A.s.fd, sp[LX] - sp[0], sp[2 * LX] - sp[-LX], sp[3 * LX] - sp[-2 * LX],
                             sp[4 * LX] - sp[-3 * LX]);
        adj_velocity_axis<N, NT>(A, D, s_tab, C, 1, y, ny, gg, L, lv, r, D1, in1, gsum);
    }
    st1<NT>(A.gs + pk, gs0 + gsum);
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

template <int N>
hipError_t adj_launch_tile2d(int which, const AdjArgs &a, size_t lds, hipStream_t s)
{
    const dim3 grid(8 * a.s.vtiles_per_xcd), block(64, a.s.plane_rows);
    if (a.s.plane_rows == 16) {
        if (which == 0)
            k_adj_pressure_tile2d<N, 16><<<grid, block, lds, s>>>(a);
        else
            k_adj_velocity_tile2d<N, 16><<<grid, block, lds, s>>>(a);
    } else if (a.s.plane_rows == 8) {
        if (which == 0)
            k_adj_pressure_tile2d<N, 8><<<grid, block, lds, s>>>(a);
        else
            k_adj_velocity_tile2d<N, 8><<<grid, block, lds, s>>>(a);
    } else {
        if (which == 0)
            k_adj_pressure_tile2d<N, 4><<<grid, dim3(64, 4), lds, s>>>(a);
        else
            k_adj_velocity_tile2d<N, 4><<<grid, dim3(64, 4), lds, s>>>(a);
    }
    return hipGetLastError();
}

template <int NDIM, int N>
hipError_t adj_launch(int which, const AdjArgs &a, hipStream_t s)
{
    // 2D with the tile kernels on: the two reverse-step kernels on their tiles
    if (NDIM == 2 && which < 2 && a.s.plane && a.s.n_vtiles > 0)
        return adj_launch_tile2d<N>(which, a, (size_t)a.s.class_cap * (2 + 4 * N) * sizeof(float), s);
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
    const float f2 = A.noise_amp != 0.0f ? speed_factor_sq(D.noise_seed, (uint32_t)g, A.noise_amp) : 1.0f;
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
