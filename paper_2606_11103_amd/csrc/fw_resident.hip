// Resident 1D step: one workgroup per 1D domain keeps the whole domain on
// the chip for a run of steps.  p and v live in LDS (with four zero cells on
// either side, the outside of the domain), the memory variables of the two
// operators in registers (strided ownership: thread t holds cells t, t + 1024,
// ...), the CPML variables of the two slabs in LDS; every step is the
// velocity update and the pressure update (with the sources and receivers of
// the cells it updates), separated by workgroup barriers, and HBM is touched
// only to load the state at the start and store it at the end of the run
// (plus the source waveforms and the receiver traces).  A 1D domain of 8192
// cells at N = 4 holds 320 KB of state: a per-step pass over HBM or the
// last-level cache costs far more than the arithmetic, so the step is kept on
// chip.
//
// Each value is computed with the operations of k_velocity / k_pressure /
// k_src_rec in 1D, in the same order (Sec. 3.3 step with the memory
// variables of Eq. (relaxation_psi), CPML in the same recursion form as the
// tissue (Sec. 2.1), sources and receivers of Sec. 4.1), so the results are
// bitwise those of the per-step kernels.
#include "fw_internal.h"
#include "fw_vec.h"

namespace fw {

namespace {

constexpr int kNT = 1024;                          // threads per workgroup
constexpr int kK = kResident1dCells / kNT;         // cells per thread

// bad_row <- min(bad_row, t) with -1 meaning "none yet"; workgroups run
// different steps at the same time, so the first row is kept by value
__device__ void flag_bad_row(int64_t *bad_row, int64_t t)
{
    unsigned long long *a = reinterpret_cast<unsigned long long *>(bad_row);
    unsigned long long cur = __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const int64_t c = (int64_t)cur;
        if (c >= 0 && c <= t) return;
        const unsigned long long prev = atomicCAS(a, cur, (unsigned long long)t);
        if (prev == cur) return;
        cur = prev;                       // another workgroup changed it: retry against its value
    }
}

// N consecutive coefficients of a class record as one LDS access (the
// record's groups of four start on 16-byte boundaries)
template <int N>
__device__ __forceinline__ void coef_group(const float *p, float (&v)[N])
{
    if constexpr (N >= 3) {
        const float4 q = *reinterpret_cast<const float4 *>(p);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        if constexpr (N == 4) v[3] = q.w;
    } else if constexpr (N == 2) {
        const float2 q = *reinterpret_cast<const float2 *>(p);
        v[0] = q.x;
        v[1] = q.y;
    } else {
        v[0] = p[0];
    }
}

template <bool B> struct BoolTag {
    static constexpr bool value = B;
};

// per-class coefficients of both operators in one LDS record per class, so
// that a cell addresses all of them from one base (class x kCoefStride)
constexpr int kCoefStride = 24;
constexpr int kIK1 = 0, kIK2 = 1, kKB = 2, kTB = 3, kA1 = 4, kB1 = 8, kA2 = 12, kB2 = 16, kRHO = 20;

template <int N>
__global__ __launch_bounds__(kNT) void k_resident1d(const Resident1dArgs R)
{
    constexpr int L0 = 4;                             // LDS index of cell 0
    __shared__ float sp[kResident1dCells + 8];
    __shared__ float sv[kResident1dCells + 8];
    __shared__ uint8_t scl[kResident1dCells];
    // CPML of the slab cells (slab index: [0, P) the first slab, [P, 2P) the
    // last): memory variables and coefficients of both operators
    __shared__ float spp1[kResident1dSlab], spp2[kResident1dSlab];
    __shared__ float saF[kResident1dSlab], sbF[kResident1dSlab], saC[kResident1dSlab], sbC[kResident1dSlab];
    // per cell: its entry in the domain's source/receiver list (-1: none), so
    // the thread that updates a cell's pressure also injects its source and
    // records its receivers, with no separate pass and barrier
    __shared__ int16_t s_sr[kResident1dCells];
    __shared__ int s_last, s_mixed;
    extern __shared__ __align__(16) float s_coef[];    // [class][kCoefStride], 16-byte aligned records
    const StepArgs &A = R.s;

    const int d = blockIdx.x;
    const int tid = threadIdx.x;
    const DomainDesc D = A.doms[d];
    const int n = (int)D.n[0];
    const int P = A.pml;
    const int ns = 2 * P < n ? 2 * P : n;             // slab cells: [0, P) and [n - P, n)
    const int64_t o = D.cell_off;
    const int64_t t0 = *R.step;
    const int32_t poff = D.pml_off[0];

    for (int c = tid; c < D.n_classes; c += kNT) {
        const ClassCoef &cc = A.classes[D.class_base + c];
        float *r = s_coef + c * kCoefStride;
        r[kIK1] = cc.ik1;
        r[kIK2] = cc.ik2;
        r[kKB] = cc.K;
        r[kTB] = cc.twobeta;
        r[kRHO] = cc.rho;
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            r[kA1 + nu] = cc.a1[nu];
            r[kB1 + nu] = cc.b1[nu];
            r[kA2 + nu] = cc.a2[nu];
            r[kB2 + nu] = cc.b2[nu];
        }
    }
    for (int i = tid; i < kResident1dCells + 8; i += kNT) {
        sp[i] = 0.0f;
        sv[i] = 0.0f;
    }
    if (tid == 0) s_mixed = 0;
    __syncthreads();
    for (int i = tid; i < n; i += kNT) {
        sp[L0 + i] = A.f.p[o + i];
        sv[L0 + i] = A.f.vx[o + i];
        scl[i] = A.f.cls[o + i];
    }
    for (int s = tid; s < ns; s += kNT) {
        const int i = s < P ? s : n - 2 * P + s;
        spp1[s] = A.f.pP1[0][o + i];
        spp2[s] = A.f.pP2[0][o + i];
        saF[s] = A.pml_tab[poff + i];
        sbF[s] = A.pml_tab[poff + n + i];
        saC[s] = A.pml_tab[poff + 2 * n + i];
        sbC[s] = A.pml_tab[poff + 3 * n + i];
    }
    float ps1[kK][N], ps2[kK][N], mf[kK], Kf[kK];
    int cb[kK];                                       // LDS record of the cell's class
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const int i = tid + k * kNT;
        if (i < n) {
            load_stream<N>(A.f.psi1x + (o + i) * N, ps1[k]);
            load_stream<N>(A.f.psi2 + (o + i) * N, ps2[k]);
        }
    }
    __syncthreads();
    // a domain of one class (a homogeneous medium: every domain of an
    // attenuation sweep) reads its coefficients once, into scalar registers
    for (int i = tid; i < n; i += kNT)
        if (scl[i] != scl[0]) s_mixed = 1;
    // per-cell constants of the run: class record, face coefficient
    // 2 dt / (rho_i + rho_{i+1}) and the (perturbed) bulk modulus, formed as
    // the step kernels form them
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const int i = tid + k * kNT;
        cb[k] = 0;
        mf[k] = 0.0f;
        Kf[k] = 0.0f;
        if (i < n) {
            const int L = scl[i];
            const int Ln = (i + 1 < n) ? scl[i + 1] : L;
            cb[k] = L * kCoefStride;
            mf[k] = 2.0f * A.dt / (s_coef[L * kCoefStride + kRHO] + s_coef[Ln * kCoefStride + kRHO]);
            float K = s_coef[L * kCoefStride + kKB];
            if (A.noise_amp != 0.0f) K = K * speed_factor_sq(D.noise_seed, (uint32_t)i, A.noise_amp);
            Kf[k] = K;
        }
    }
    // no range table: no source or receiver has been set
    const int32_t sr0 = R.sr_range ? R.sr_range[d] : 0, sr1 = R.sr_range ? R.sr_range[d + 1] : 0;
    for (int i = tid; i < n; i += kNT) s_sr[i] = -1;
    __syncthreads();
    for (int32_t e = sr0 + tid; e < sr1; e += kNT) s_sr[(int)(R.cells[e].cell - o)] = (int16_t)(e - sr0);
    __syncthreads();
    // one class and no speed perturbation: every coefficient of the step,
    // the face coefficient and the bulk modulus included, is the same in
    // every cell of the domain
    const bool uniform = s_mixed == 0 && A.noise_amp == 0.0f;
    // the run's steps; with UNI every cell's coefficients are those of the
    // domain's single class (same values as the per-cell path reads)
    // (readfirstlane takes lane 0's value: a wave with work always has cell
    // tid < n in lane 0, so its per-cell constants are set)
    auto run = [&](auto uni_tag) {
    constexpr bool UNI = decltype(uni_tag)::value;
    const int Lu = n > 0 ? scl[0] * kCoefStride : 0;
    auto sgpr = [](float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); };
    float u_ik1 = 0.0f, u_ik2 = 0.0f, u_tb = 0.0f, u_mf = 0.0f, u_K = 0.0f, u_a1[N], u_b1[N], u_a2[N], u_b2[N];
    if constexpr (UNI) {
        u_mf = sgpr(mf[0]);
        u_K = sgpr(Kf[0]);
        u_ik1 = sgpr(s_coef[Lu + kIK1]);
        u_ik2 = sgpr(s_coef[Lu + kIK2]);
        u_tb = sgpr(s_coef[Lu + kTB]);
#pragma unroll
        for (int nu = 0; nu < N; ++nu) {
            u_a1[nu] = sgpr(s_coef[Lu + kA1 + nu]);
            u_b1[nu] = sgpr(s_coef[Lu + kB1 + nu]);
            u_a2[nu] = sgpr(s_coef[Lu + kA2 + nu]);
            u_b2[nu] = sgpr(s_coef[Lu + kB2 + nu]);
        }
    }
    for (int st = 0; st < R.n_steps; ++st) {
        const int64_t t = t0 + st;
        // the thread index passes through an empty asm statement each step, so
        // the compiler forms the per-cell LDS addresses inside the loop (a few
        // integer operations) instead of holding all of them across it
        int tb = tid;
        asm volatile("" : "+v"(tb));
        // velocity update: reads p (stencil) and the thread's own v
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            const int i = tb + k * kNT;
            if (i >= n) continue;
            const float *sr = sp + L0 + i;
            float Da = stencil4(A.fd, sr[1] - sr[0], sr[2] - sr[-1], sr[3] - sr[-2], sr[4] - sr[-3]);
            if (i < P || i >= n - P) {
                const int s = i < P ? i : i - n + 2 * P;
                const float qv = fmaf(saF[s], Da, sbF[s] * spp1[s]);
                spp1[s] = qv;
                Da += qv;
            }
            const float *cr = s_coef + cb[k];
            float ca[N], cbv[N];
            if constexpr (!UNI) {
                coef_group<N>(cr + kA1, ca);
                coef_group<N>(cr + kB1, cbv);
            }
            float sacc = (UNI ? u_ik1 : cr[kIK1]) * Da;
#pragma unroll
            for (int nu = 0; nu < N; ++nu) {
                const float a = UNI ? u_a1[nu] : ca[nu], b = UNI ? u_b1[nu] : cbv[nu];
                ps1[k][nu] = fmaf(1.0f * a, Da, b * ps1[k][nu]);
                sacc += ps1[k][nu];
            }
            sv[L0 + i] = fmaf(-(UNI ? u_mf : mf[k]), sacc, sv[L0 + i]);
        }
        __syncthreads();
        // pressure update: reads v (stencil) and the thread's own p
        asm volatile("" : "+v"(tb));
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            const int i = tb + k * kNT;
            if (i >= n) continue;
            const float *sx = sv + L0 + i;
            float S = stencil4(A.fd, sx[0] - sx[-1], sx[1] - sx[-2], sx[2] - sx[-3], sx[3] - sx[-4]);
            if (i < P || i >= n - P) {
                const int s = i < P ? i : i - n + 2 * P;
                const float qv = fmaf(saC[s], S, sbC[s] * spp2[s]);
                spp2[s] = qv;
                S += qv;
            }
            const float *cr = s_coef + cb[k];
            float ca[N], cbv[N];
            if constexpr (!UNI) {
                coef_group<N>(cr + kA2, ca);
                coef_group<N>(cr + kB2, cbv);
            }
            float Tt = (UNI ? u_ik2 : cr[kIK2]) * S;
#pragma unroll
            for (int nu = 0; nu < N; ++nu) {
                const float a = UNI ? u_a2[nu] : ca[nu], b = UNI ? u_b2[nu] : cbv[nu];
                ps2[k][nu] = fmaf(1.0f * a, S, b * ps2[k][nu]);
                Tt += ps2[k][nu];
            }
            const float pn0 = sp[L0 + i];
            float v = fmaf(-(A.dt * fmaf(UNI ? u_tb : cr[kTB], pn0, UNI ? u_K : Kf[k])), Tt, pn0);
            const int es = s_sr[i];
            if (es >= 0) {
                // the cell's source, then its receivers (after the injection)
                const SrcRecCell c = R.cells[sr0 + es];
                if (t < R.n_t && c.wave >= 0) v += R.waves[(int64_t)c.wave * R.n_t + t];
                if (t < R.n_t_max) {
                    for (int32_t q = c.r0; q < c.r1; ++q) R.traces[t * R.n_rec + R.rec_of[q]] = v;
                    if (c.r1 > c.r0 && !isfinite(v)) flag_bad_row(R.bad_row, t);
                }
            }
            sp[L0 + i] = v;
        }
        __syncthreads();
    }
    };
    // (at N >= 3 the coefficients held in registers would not fit beside the
    // memory variables: those domains take the per-cell path)
    if (N <= 2 && uniform)
        run(BoolTag<N <= 2>{});
    else
        run(BoolTag<false>{});

    // store the state of the run's last step
    for (int i = tid; i < n; i += kNT) {
        A.fo.p[o + i] = sp[L0 + i];
        A.fo.vx[o + i] = sv[L0 + i];
    }
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const int i = tid + k * kNT;
        if (i < n) {
            store_stream<N>(A.fo.psi1x + (o + i) * N, ps1[k]);
            store_stream<N>(A.fo.psi2 + (o + i) * N, ps2[k]);
        }
    }
    for (int s = tid; s < ns; s += kNT) {
        const int i = s < P ? s : n - 2 * P + s;
        A.fo.pP1[0][o + i] = spp1[s];
        A.fo.pP2[0][o + i] = spp2[s];
    }
    // the last workgroup to finish advances the step counter (every
    // workgroup has read it by then) and re-arms the count
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        s_last = atomicAdd(R.done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && tid == 0) {
        *R.done = 0u;
        *R.step = t0 + R.n_steps;
    }
}

}  // namespace

size_t resident1d_lds_bytes(int nmech, int class_cap)
{
    (void)nmech;
    return (size_t)kCoefStride * class_cap * sizeof(float);
}

hipError_t launch_resident1d(int nmech, const Resident1dArgs &r, int n_domains, hipStream_t s)
{
    const size_t lds = resident1d_lds_bytes(nmech, r.s.class_cap);
    const dim3 grid((unsigned)n_domains), block(kNT);
    switch (nmech) {
    case 1: k_resident1d<1><<<grid, block, lds, s>>>(r); break;
    case 2: k_resident1d<2><<<grid, block, lds, s>>>(r); break;
    case 3: k_resident1d<3><<<grid, block, lds, s>>>(r); break;
    case 4: k_resident1d<4><<<grid, block, lds, s>>>(r); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fw
