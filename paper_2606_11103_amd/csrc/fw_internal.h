// Internal types shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fw {

constexpr int kMaxMech = 4;
constexpr int kMaxLocalClasses = 256;   // class indices are uint8 within a domain

// FP32 per-class coefficients, produced on the host in FP64 and rounded once.
struct ClassCoef {
    float ik1;        // 1 / kappa_1 (gradient operator)
    float ik2;        // 1 / kappa_2 (divergence operator)
    float rho;        // density
    float K;          // bulk modulus rho c^2 (without the per-voxel perturbation)
    float twobeta;    // 2 beta of the pressure-dependent modulus K + 2 beta p
    float pad[3];
    float a1[kMaxMech], b1[kMaxMech];   // recursion coefficients, gradient operator
    float a2[kMaxMech], b2[kMaxMech];   // recursion coefficients, divergence operator
};

struct DomainDesc {
    int64_t n[3];          // nx, ny, nz
    int64_t cell_off;      // first cell of the domain in the concatenated arrays
    int32_t class_base;    // first global class of the domain
    int32_t n_classes;     // number of local classes
    int32_t pml_off[3];    // offset of the per-axis CPML tables [aF|bF|aC|bC] x n[a]
    int32_t pitch;         // row stride in cells: nx rounded up to 32 cells (128 B) in 2D/3D, nx in 1D;
                           // cell (x, y, z) is stored at cell_off + (z*ny + y)*pitch + x
    uint64_t noise_seed;
    int64_t packed_off;    // first cell of the domain in the unpadded (caller) layout
};

// A tile: a block of cells along x (and y in 3D) marched over [z0, z1) of
// the marching axis (z in 3D, y in 2D, a single row in 1D).
struct Tile {
    int32_t dom, x0, y0, z0, z1, pad0, pad1, pad2;
};

struct Fields {
    float *p, *vx, *vy, *vz;
    float *psi1x, *psi1y, *psi1z;   // [cell][N] gradient-operator memory variables per axis
    float *psi2;                    // [cell][N] divergence-operator memory variables, summed over axes
    float *pP1[3], *pP2[3];         // CPML memory variables per axis (touched inside slabs only)
    uint8_t *cls;
};

struct StepArgs {
    Fields f;                  // state read by the step
    Fields fo;                 // state written by the step (== f: in place)
    const DomainDesc *doms;
    const Tile *tiles;
    const ClassCoef *classes;
    const float *pml_tab;
    int32_t n_tiles;
    int32_t tiles_per_xcd;     // ceil(n_tiles / 8): XCD x owns tiles [x C, (x + 1) C)
    int32_t blocks_per_xcd;    // blocks per XCD of the step kernels (= tiles_per_xcd, or fewer: persistent)
    int32_t pml;               // CPML width P
    int32_t class_cap;         // entries per LDS class table (>= classes of any domain)
    int32_t tile_rows;         // rows of a 3D tile along y
    int32_t plane;             // 1: the velocity update runs its plane kernel (2D: tile kernel) on vtiles
    int32_t plane_p;           // 1: the pressure update runs its plane kernel (2D: tile kernel) on ptiles
    int32_t plane_rows;        // rows of the plane kernels' tiles (3D: 4 or 8; 2D tile kernels: 4, 8 or 16)
    int32_t vel_planes;        // planes per velocity plane-kernel tile (1, 2 or 4)
    int32_t prs_planes;        // planes per pressure plane-kernel tile (2, 4 or 8)
    const Tile *vtiles;        // velocity (2D: also the adjoint's tiles): 64 x plane_rows tiles of vel_planes planes,
                               // plane-major, XCD k owning y-band k
    int32_t n_vtiles;
    int32_t vtiles_per_xcd;
    const Tile *ptiles;        // pressure: 64 x plane_rows tiles of prs_planes planes, same banding
    int32_t n_ptiles;
    int32_t ptiles_per_xcd;
    float fd[4];               // staggered coefficients c_m / dx
    float fd_b;                // off-axis weight b / dx of the widened 2D stencil (0: on-axis only)
    float dt;
    float noise_amp;
    // optional per-voxel relaxation strength scale s(x) in [0, 1] (NULL: 1
    // everywhere), unpadded layout (DomainDesc::packed_off + local index):
    // the memory-variable coefficients a of both operators are multiplied by s
    const float *amap;
};

// One distinct source or receiver cell: the waveform row of its source (-1:
// none; a cell holds at most one source) and its receivers, entries
// [r0, r1) of the grouped list.
struct SrcRecCell {
    int64_t cell;              // global cell index
    int32_t wave, r0, r1, pad;
};

struct SrcRecArgs {
    float *p;
    const SrcRecCell *cells;   // distinct source/receiver cells, sorted by cell
    int64_t n_cells;
    const int32_t *rec_of;     // receiver indices grouped by cell
    const float *waves;        // [n_wave][n_t]
    int32_t n_t;
    float *traces;             // [n_t_max][n_rec]
    int64_t n_rec;
    int32_t n_t_max;
    int64_t *step;             // device step counter
    int64_t *bad_row;          // first trace row holding a non-finite value, -1 if none
    uint32_t *done;            // workgroups finished in this launch (0 between launches)
};

// d a / d s and d b / d s per mechanism when d -> s d (adjoint gradients)
struct ClassAdj {
    float a1s[kMaxMech], b1s[kMaxMech], a2s[kMaxMech], b2s[kMaxMech];
};

struct AdjArgs {
    StepArgs s;                // tables, tiles and the forward state u^n (s.f)
    Fields fnext;              // forward state u^{n+1}
    Fields lam;                // adjoint state (same layout as the forward state)
    float *lamD1[3], *lamD2[3];
    float *gK, *gs;            // gradients, unpadded layout
    const ClassAdj *cadj;
    int32_t tile_rows;
    int32_t fold_div;          // 1: lamD1 holds the previous reverse step's
                               //    velocity output, still to be applied to lam_p
};

struct AdjInjectArgs {
    float *lam_p;
    const int64_t *cells;      // distinct receiver cells (global index)
    const int32_t *offsets;    // [n_cells + 1] into rec_index
    const int32_t *rec_index;  // receivers grouped by cell
    int64_t n_cells;
    const float *res;          // [n_steps][n_rec] dJ/d trace
    int64_t n_rec;
    int64_t step;
};

// Chain rule of the adjoint from the modulus and d-scale gradients to the
// gradients of the sound speed and of the attenuation coefficient alpha0:
//   dJ/dc(x)      = 2 rho c (1 + eps(x))^2 dJ/dK(x)   (K = rho c^2 (1 + eps)^2),
//   dJ/dalpha0(x) = dJ/ds(x) / alpha0                 (d proportional to alpha0),
// with rho, c, alpha0 of the cell's class and eps its speed perturbation.
struct AdjChainArgs {
    const DomainDesc *doms;
    int32_t n_domains;
    float noise_amp;
    const uint8_t *cls;        // class map (padded layout: doms[d].cell_off + local index)
    const float2 *chain;       // per global class: (2 rho c, 1 / alpha0)
    const float *gK, *gs;      // dJ/dK, dJ/ds in the unpadded layout
    float *grad_c, *grad_a0;   // accumulated (+=), unpadded layout; grad_a0 may be NULL
    int64_t n_packed;
};

// Resident 1D step (fw_resident.hip): one workgroup per 1D domain of at most
// kResident1dCells cells keeps the domain's state on chip for n_steps steps
// (velocity, pressure, sources/receivers of each step), for CPML widths up to
// kResident1dSlab / 2 cells.
constexpr int kResident1dCells = 8192;
constexpr int kResident1dSlab = 1024;

struct Resident1dArgs {
    StepArgs s;                // fields (read from s.f, written to s.fo), domains, tables, dt, noise
    const SrcRecCell *cells;   // distinct source/receiver cells, sorted by cell
    const int32_t *sr_range;   // [n_domains + 1]: domain d's entries of cells are [sr_range[d], sr_range[d + 1])
    const int32_t *rec_of;
    const float *waves;
    int32_t n_t;
    float *traces;
    int64_t n_rec;
    int32_t n_t_max;
    int32_t n_steps;
    int64_t *step, *bad_row;
    uint32_t *done;
};

size_t resident1d_lds_bytes(int nmech, int class_cap);
hipError_t launch_resident1d(int nmech, const Resident1dArgs &r, int n_domains, hipStream_t s);

hipError_t launch_copy(void *dst, const void *src, int64_t bytes, hipStream_t s);
// memory-traffic probe of one 3D domain: mode 0 velocity streams, 1 pressure
// streams, 2 both in one pass; order 0 flat sweep, 1 64 x 4 tiles marching 48 planes
hipError_t launch_stream_probe(int nmech, int mode, int order, const Fields &F, int64_t nx, int64_t px, int64_t ny,
                               int64_t nz, hipStream_t s);
// *count += number of the n values that are not finite numbers in [0, 1]
hipError_t launch_count_outside_unit(const float *x, int64_t n, unsigned long long *count, hipStream_t s);
hipError_t launch_adjoint_chain(const AdjChainArgs &a, hipStream_t s);
hipError_t launch_energy(int ndim, const StepArgs &a, const float *p_old, double *partial, hipStream_t s);
// one reverse step: transpose of the pressure update (applying a pending
// lamD1 first when a.fold_div is set), then of the velocity update
hipError_t launch_adjoint_step(int ndim, int nmech, const AdjArgs &a, hipStream_t s);
// lam_p -= sum_a div_a(lamD1_a): completes the last reverse step
hipError_t launch_adjoint_finish(int ndim, const AdjArgs &a, hipStream_t s);
hipError_t launch_adjoint_inject(const AdjInjectArgs &a, hipStream_t s);

// Launchers (kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_velocity(int ndim, int nmech, int tile_rows, int rows_per_thread, const StepArgs &a, hipStream_t s);
hipError_t launch_pressure(int ndim, int nmech, int tile_rows, int rows_per_thread, const StepArgs &a, hipStream_t s);
hipError_t launch_src_rec(const SrcRecArgs &a, hipStream_t s);
// Tile footprint of a launch configuration: cells per tile along x and y.
void tile_shape(int ndim, int tile_rows, int *tx, int *ty);

}  // namespace fw
