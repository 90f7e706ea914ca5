/*
 * FP64 reference solver for the attenuating, nonlinear acoustic FDTD step.
 *
 * TEST INFRASTRUCTURE: this is the oracle.  Only tests/, the smoke() check and
 * the cpu_baseline leg of bench.py may build, load or call it.  It shares no
 * code, header, table or constant with the product library.
 *
 * What it computes (paper Sec. 2.1 and Sec. 3.3), literally and unfused:
 *   - the stretched pressure-velocity system, Eqs. (wave1) and (wave2):
 *       rho dv/dt = -d~p/dx~ ,  kappa dp/dt = -div~ v   (kappa = 1/K),
 *   - the stretched derivative of Eq. (relaxation4): d/dx~ = (1/kappa_i) d/dx
 *     + sum_nu psi_i^nu, with one memory variable per axis, per operator
 *     (i = 1 for the gradient, i = 2 for the divergence) and per mechanism,
 *   - the recursion of Eq. (relaxation_psi), psi <- b psi + a D, updated with
 *     the derivative of the same sub-step and then used ("update, then use"),
 *   - one more memory variable per axis for the CPML, same recursion form,
 *     applied to the tissue-stretched derivative: the CPML stretches the
 *     coordinate of the lossy medium, so the two stretch factors multiply
 *     (d/dx~ = (1/s_pml)(1/s_tissue) d/dx), which keeps the layer
 *     reflectionless and stable for any tissue,
 *   - a pressure-dependent bulk modulus K + 2 beta p for the nonlinearity,
 *   - the 2M-th order staggered stencil (M = 4) with leapfrog time stepping.
 * Every per-voxel coefficient arrives as its own FP64 array; nothing is
 * summed across axes, cached or fused.  Values outside the grid are zero.
 *
 * Layout: x fastest, then y, then z; linear index (k*ny + j)*nx + i.
 * The face "i+1/2" along an axis is stored at the index of cell i.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t ndim, nmech;
    int64_t n[3];
    double dx, dt;
    double fd[4];                      /* staggered coefficients c_1..c_4 */
    double fd_b;                       /* off-axis weight (0: on-axis stencil only) */
    /* per-cell material arrays [cells] */
    const double *rho, *K, *beta, *ik1, *ik2;
    /* per-cell recursion coefficients [nmech][cells] */
    const double *a1, *b1, *a2, *b2;
    /* CPML profiles along each axis, [3][nmax]: faces (F) and cells (C) */
    const double *pml_aF, *pml_bF, *pml_aC, *pml_bC;
    int64_t nmax;
    /* state, caller-owned */
    double *p;                         /* [cells]              */
    double *v;                         /* [3][cells]           */
    double *psi1;                      /* [3][nmech][cells]    */
    double *psi2;                      /* [3][nmech][cells]    */
    double *psiP1, *psiP2;             /* [3][cells]           */
} ora_sim;

static int64_t ncells(const ora_sim *s) { return s->n[0] * s->n[1] * s->n[2]; }

static int64_t stride_of(const ora_sim *s, int a)
{
    return a == 0 ? 1 : (a == 1 ? s->n[0] : s->n[0] * s->n[1]);
}

static int64_t coord_of(const ora_sim *s, int64_t idx, int a)
{
    if (a == 0) return idx % s->n[0];
    if (a == 1) return (idx / s->n[0]) % s->n[1];
    return idx / (s->n[0] * s->n[1]);
}

/* Off-axis part of the axis-a difference (the widened stencil of Tan and
 * Huang): the two-point difference f[ia + hi] - f[ia + lo] along axis a taken
 * in the rows one cell away along every other axis o, both sides, summed;
 * zero outside the grid.  The gradient at face i+1/2 uses (hi, lo) = (1, 0),
 * the divergence at cell i uses (0, -1). */
static double off_axis(const ora_sim *s, const double *f, int64_t idx, int a, int hi, int lo)
{
    if (s->fd_b == 0.0) return 0.0;
    const int64_t st = stride_of(s, a), ia = coord_of(s, idx, a), na = s->n[a];
    double acc = 0.0;
    for (int o = 0; o < s->ndim; ++o) {
        if (o == a) continue;
        const int64_t so = stride_of(s, o), io = coord_of(s, idx, o), no = s->n[o];
        for (int sg = -1; sg <= 1; sg += 2) {
            const int64_t jo = io + sg;
            if (jo < 0 || jo >= no) continue;
            const int64_t row = idx + sg * so;
            const double fh = (ia + hi >= 0 && ia + hi < na) ? f[row + hi * st] : 0.0;
            const double fl = (ia + lo >= 0 && ia + lo < na) ? f[row + lo * st] : 0.0;
            acc += fh - fl;
        }
    }
    return acc;
}

/* Staggered gradient of a cell field f at face i+1/2 of axis a:
 * (1/dx) sum_m c_m (f[i+m] - f[i+1-m]), zero outside the grid. */
static double grad_face(const ora_sim *s, const double *f, int64_t idx, int a)
{
    const int64_t st = stride_of(s, a), ia = coord_of(s, idx, a), na = s->n[a];
    double D = 0.0;
    for (int m = 1; m <= 4; ++m) {
        const int64_t jp = ia + m, jm = ia + 1 - m;
        const double fp = (jp >= 0 && jp < na) ? f[idx + (jp - ia) * st] : 0.0;
        const double fm = (jm >= 0 && jm < na) ? f[idx + (jm - ia) * st] : 0.0;
        D += s->fd[m - 1] * (fp - fm);
    }
    D += s->fd_b * off_axis(s, f, idx, a, 1, 0);
    return D / s->dx;
}

/* Staggered divergence term of a face field g at cell i along axis a:
 * (1/dx) sum_m c_m (g[i+m-1] - g[i-m]), zero outside the grid. */
static double div_cell(const ora_sim *s, const double *g, int64_t idx, int a)
{
    const int64_t st = stride_of(s, a), ia = coord_of(s, idx, a), na = s->n[a];
    double D = 0.0;
    for (int m = 1; m <= 4; ++m) {
        const int64_t jp = ia + m - 1, jm = ia - m;
        const double gp = (jp >= 0 && jp < na) ? g[idx + (jp - ia) * st] : 0.0;
        const double gm = (jm >= 0 && jm < na) ? g[idx + (jm - ia) * st] : 0.0;
        D += s->fd[m - 1] * (gp - gm);
    }
    D += s->fd_b * off_axis(s, g, idx, a, 0, -1);
    return D / s->dx;
}

/* Face density: mean of the two cells that share the face; the last face of
 * an axis has no right neighbour and takes the density of its owner cell. */
static double rho_face(const ora_sim *s, int64_t idx, int a)
{
    const int64_t st = stride_of(s, a), ia = coord_of(s, idx, a);
    const double rl = s->rho[idx];
    const double rr = (ia + 1 < s->n[a]) ? s->rho[idx + st] : rl;
    return 0.5 * (rl + rr);
}

/* Velocity sub-step: gradient, memory variables of operator 1, CPML. */
static void step_velocity(ora_sim *s)
{
    const int64_t nc = ncells(s);
    for (int a = 0; a < s->ndim; ++a) {
        double *va = s->v + (int64_t)a * nc;
        double *psiP = s->psiP1 + (int64_t)a * nc;
        const double *aF = s->pml_aF + (int64_t)a * s->nmax;
        const double *bF = s->pml_bF + (int64_t)a * s->nmax;
#pragma omp parallel for schedule(static)
        for (int64_t idx = 0; idx < nc; ++idx) {
            const double D = grad_face(s, s->p, idx, a);
            double sum = s->ik1[idx] * D;
            for (int nu = 0; nu < s->nmech; ++nu) {
                const int64_t o = ((int64_t)a * s->nmech + nu) * nc + idx;
                const int64_t c = (int64_t)nu * nc + idx;
                s->psi1[o] = s->b1[c] * s->psi1[o] + s->a1[c] * D;
                sum += s->psi1[o];
            }
            const int64_t ia = coord_of(s, idx, a);
            psiP[idx] = bF[ia] * psiP[idx] + aF[ia] * sum;
            sum += psiP[idx];
            va[idx] -= s->dt / rho_face(s, idx, a) * sum;
        }
    }
}

/* Pressure sub-step: divergence, memory variables of operator 2, CPML and
 * the pressure-dependent modulus K + 2 beta p (explicit in p^n). */
static void step_pressure(ora_sim *s)
{
    const int64_t nc = ncells(s);
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < nc; ++idx) {
        double T = 0.0;
        for (int a = 0; a < s->ndim; ++a) {
            const double D = div_cell(s, s->v + (int64_t)a * nc, idx, a);
            double term = s->ik2[idx] * D;
            for (int nu = 0; nu < s->nmech; ++nu) {
                const int64_t o = ((int64_t)a * s->nmech + nu) * nc + idx;
                const int64_t c = (int64_t)nu * nc + idx;
                s->psi2[o] = s->b2[c] * s->psi2[o] + s->a2[c] * D;
                term += s->psi2[o];
            }
            const int64_t ia = coord_of(s, idx, a);
            double *psiP = s->psiP2 + (int64_t)a * nc;
            psiP[idx] = s->pml_bC[a * s->nmax + ia] * psiP[idx] + s->pml_aC[a * s->nmax + ia] * term;
            term += psiP[idx];
            T += term;
        }
        const double pn = s->p[idx];
        s->p[idx] = pn - s->dt * (s->K[idx] + 2.0 * s->beta[idx] * pn) * T;
    }
}

/* Staggered-time energy E^{n+1/2} = 1/2 sum rho_f |v^{n+1/2}|^2
 * + 1/2 sum p^{n+1} p^n / K, summed plane by plane in a fixed order. */
static double energy(const ora_sim *s, const double *p_old)
{
    const int64_t nc = ncells(s);
    const int64_t plane = s->n[0] * s->n[1];
    const int64_t nz = s->n[2];
    double *part = (double *)calloc((size_t)nz, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k) {
        double acc = 0.0;
        for (int64_t q = 0; q < plane; ++q) {
            const int64_t idx = k * plane + q;
            acc += 0.5 * s->p[idx] * p_old[idx] / s->K[idx];
            for (int a = 0; a < s->ndim; ++a) {
                const double va = s->v[(int64_t)a * nc + idx];
                acc += 0.5 * rho_face(s, idx, a) * va * va;
            }
        }
        part[k] = acc;
    }
    double E = 0.0;
    for (int64_t k = 0; k < nz; ++k) E += part[k];
    free(part);
    return E;
}

/*
 * Advance n_steps steps.  Step number t (0-based, counted from step0) adds
 * src_wave[s][t] to p at src_cell[s] after the pressure update (additive soft
 * source, t < n_t only) and then records rec_out[t-step0... local][r] =
 * p[rec_cell[r]].  energy_out (may be NULL) receives E^{n+1/2} per step.
 * Returns 0, or -1 on a non-finite pressure at a receiver.
 */
int oracle_steps(ora_sim *s, int n_steps, int step0,
                 int64_t n_src, const int64_t *src_cell, const double *src_wave, int n_t,
                 int64_t n_rec, const int64_t *rec_cell, double *rec_out, double *energy_out)
{
    const int64_t nc = ncells(s);
    double *p_old = NULL;
    if (energy_out) p_old = (double *)malloc((size_t)nc * sizeof(double));
    int status = 0;
    for (int t = 0; t < n_steps; ++t) {
        const int step = step0 + t;
        step_velocity(s);
        if (p_old) memcpy(p_old, s->p, (size_t)nc * sizeof(double));
        step_pressure(s);
        if (step < n_t)
            for (int64_t q = 0; q < n_src; ++q)
                s->p[src_cell[q]] += src_wave[q * (int64_t)n_t + step];
        for (int64_t r = 0; r < n_rec; ++r) {
            const double val = s->p[rec_cell[r]];
            if (!isfinite(val)) status = -1;
            if (rec_out) rec_out[(int64_t)t * n_rec + r] = val;
        }
        if (energy_out) energy_out[t] = energy(s, p_old);
    }
    free(p_old);
    return status;
}

/* ------------------------------------------------------------------------
 * Discrete adjoint of one linear step (beta = 0), literal per axis.
 *
 * The forward step maps u^n = (p, v, psi1, psiP1, psi2, psiP2) to u^{n+1}.
 * Given the adjoint lam^{n+1} of u^{n+1} (in lam_*, overwritten with lam^n)
 * and the forward state u^n (in s, left unchanged), this applies the
 * transpose of the step and accumulates
 *   gK[x] += lam_p^{n+1}[x] * dp^{n+1}[x]/dK[x] = lam_p^{n+1} * (-dt T^n)
 *   gs[x] += sum over the recursions owned by x of mu * (b_s psi + a_s D)
 * where s is a per-cell scale of every d coefficient (d -> s d) and
 * a_s, b_s = da/ds, db/ds at s = 1 arrive per cell in [nmech][cells].
 * The transposes of the staggered operators follow from
 * div = -grad^T (summation by parts with zero values outside the grid).
 * ---------------------------------------------------------------------- */
int oracle_adjoint_step(ora_sim *s,
                        double *lam_p, double *lam_v, double *lam_psi1, double *lam_psiP1,
                        double *lam_psi2, double *lam_psiP2,
                        const double *a1s, const double *b1s, const double *a2s, const double *b2s,
                        double *gK, double *gs)
{
    const int64_t nc = ncells(s);
    const int nd = s->ndim, nm = s->nmech;
    /* forward intermediates of this step */
    double *D1 = (double *)malloc(sizeof(double) * nc * nd);
    double *vnew = (double *)malloc(sizeof(double) * nc * nd);
    double *D2 = (double *)malloc(sizeof(double) * nc * nd);
    double *T = (double *)malloc(sizeof(double) * nc);
    double *lamD2 = (double *)malloc(sizeof(double) * nc * nd);
    double *lamD1 = (double *)malloc(sizeof(double) * nc * nd);
    double *q = (double *)malloc(sizeof(double) * nc);
    if (!D1 || !vnew || !D2 || !T || !lamD2 || !lamD1 || !q) return -2;

    /* forward recomputation: D1, v^{n+1/2}, D2, T */
    for (int a = 0; a < nd; ++a) {
#pragma omp parallel for schedule(static)
        for (int64_t idx = 0; idx < nc; ++idx) {
            const double D = grad_face(s, s->p, idx, a);
            D1[(int64_t)a * nc + idx] = D;
            double sum = s->ik1[idx] * D;
            for (int nu = 0; nu < nm; ++nu) {
                const int64_t o = ((int64_t)a * nm + nu) * nc + idx, c = (int64_t)nu * nc + idx;
                sum += s->b1[c] * s->psi1[o] + s->a1[c] * D;
            }
            const int64_t ia = coord_of(s, idx, a);
            sum += s->pml_bF[a * s->nmax + ia] * s->psiP1[(int64_t)a * nc + idx] + s->pml_aF[a * s->nmax + ia] * sum;
            vnew[(int64_t)a * nc + idx] = s->v[(int64_t)a * nc + idx] - s->dt / rho_face(s, idx, a) * sum;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < nc; ++idx) {
        double Tx = 0.0;
        for (int a = 0; a < nd; ++a) {
            const double D = div_cell(s, vnew + (int64_t)a * nc, idx, a);
            D2[(int64_t)a * nc + idx] = D;
            double term = s->ik2[idx] * D;
            for (int nu = 0; nu < nm; ++nu) {
                const int64_t o = ((int64_t)a * nm + nu) * nc + idx, c = (int64_t)nu * nc + idx;
                term += s->b2[c] * s->psi2[o] + s->a2[c] * D;
            }
            const int64_t ia = coord_of(s, idx, a);
            term += s->pml_bC[a * s->nmax + ia] * s->psiP2[(int64_t)a * nc + idx] + s->pml_aC[a * s->nmax + ia] * term;
            Tx += term;
        }
        T[idx] = Tx;
    }

    /* transpose of the pressure sub-step */
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < nc; ++idx) {
        const double lp = lam_p[idx];
        gK[idx] += lp * (-s->dt * T[idx]);
        const double qq = -s->dt * s->K[idx] * lp;
        q[idx] = qq;
        for (int a = 0; a < nd; ++a) {
            const int64_t ia = coord_of(s, idx, a);
            /* term = Dt + psiP', psiP' = bC psiP + aC Dt: adjoint of Dt */
            const double muP = lam_psiP2[(int64_t)a * nc + idx] + qq;
            lam_psiP2[(int64_t)a * nc + idx] = s->pml_bC[a * s->nmax + ia] * muP;
            const double lDt = qq + s->pml_aC[a * s->nmax + ia] * muP;
            /* Dt = ik2 D + sum_nu psi2', psi2' = b2 psi2 + a2 D */
            double lD = s->ik2[idx] * lDt;
            for (int nu = 0; nu < nm; ++nu) {
                const int64_t o = ((int64_t)a * nm + nu) * nc + idx, c = (int64_t)nu * nc + idx;
                const double mu = lam_psi2[o] + lDt;
                lD += s->a2[c] * mu;
                gs[idx] += mu * (b2s[c] * s->psi2[o] + a2s[c] * D2[(int64_t)a * nc + idx]);
                lam_psi2[o] = s->b2[c] * mu;
            }
            lamD2[(int64_t)a * nc + idx] = lD;
        }
    }
    /* transpose of the velocity sub-step: the face adjoint first collects
     * div_a^T lamD2 = -grad_a lamD2 */
    for (int a = 0; a < nd; ++a) {
#pragma omp parallel for schedule(static)
        for (int64_t idx = 0; idx < nc; ++idx) {
            const int64_t fa = (int64_t)a * nc + idx;
            const double lv = lam_v[fa] - grad_face(s, lamD2 + (int64_t)a * nc, idx, a);
            const double r = -s->dt / rho_face(s, idx, a) * lv;
            const int64_t ia = coord_of(s, idx, a);
            /* sum = Dt + psiP', psiP' = bF psiP + aF Dt: adjoint of Dt */
            const double muP = lam_psiP1[fa] + r;
            lam_psiP1[fa] = s->pml_bF[a * s->nmax + ia] * muP;
            const double lDt = r + s->pml_aF[a * s->nmax + ia] * muP;
            /* Dt = ik1 D + sum_nu psi1', psi1' = b1 psi1 + a1 D */
            double lD = s->ik1[idx] * lDt;
            double gsum = 0.0;
            for (int nu = 0; nu < nm; ++nu) {
                const int64_t o = ((int64_t)a * nm + nu) * nc + idx, c = (int64_t)nu * nc + idx;
                const double mu = lam_psi1[o] + lDt;
                lD += s->a1[c] * mu;
                gsum += mu * (b1s[c] * s->psi1[o] + a1s[c] * D1[fa]);
                lam_psi1[o] = s->b1[c] * mu;
            }
            lamD1[fa] = lD;
            lam_v[fa] = lv;
            gs[idx] += gsum;     /* face i+1/2 is owned by cell i */
        }
    }
    /* lam_p^n = lam_p^{n+1} + sum_a grad_a^T lamD1_a = lam_p^{n+1} - sum_a div_a lamD1_a */
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < nc; ++idx) {
        double acc = 0.0;
        for (int a = 0; a < nd; ++a) acc += div_cell(s, lamD1 + (int64_t)a * nc, idx, a);
        lam_p[idx] -= acc;
    }
    free(D1); free(vnew); free(D2); free(T); free(lamD2); free(lamD1); free(q);
    return 0;
}
