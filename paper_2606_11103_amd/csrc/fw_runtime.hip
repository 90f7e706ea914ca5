// Host runtime behind the C ABI of include/fw25.h: validation, FP64 set-up of
// the per-step coefficients, workspace layout, tile lists and HIP-graph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <limits>
#include <vector>

#include "../../include/fw25.h"
#include "fw_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OR_FAIL(expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(FW_EHIP, "%s: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

// Staggered first-derivative coefficients of order 8 (Taylor construction:
// exact for odd monomials up to x^7 on the half-integer stencil).
constexpr double kFD[4] = {1225.0 / 1024.0, -245.0 / 3072.0, 49.0 / 5120.0, -5.0 / 7168.0};

// Time-space-domain staggered coefficients for the Courant number r: the
// solution of sum_m c_m (2m - 1)^(2k - 1) = r^(2k - 2), k = 1..4, which makes
// the 1D leapfrog dispersion relation sin(w dt / 2) = r sum_m c_m sin((2m - 1)
// k dx / 2) agree with w = c k through (k dx)^7 at the speed r dx / dt, so the
// step is of order 8 in time as well as in space there (Liu and Sen 2011).
// r = 0 gives the Taylor set.  Gaussian elimination with partial pivoting
// in FP64 on the 4 x 4 system of odd moments.
// shift: the widened 2D stencil's moments r^(2k - 2) - shift, shift = 2 b.
static void time_space_coefficients(double r, double out[4], double shift = 0.0)
{
    double A[4][5];
    for (int k = 0; k < 4; ++k) {
        for (int m = 0; m < 4; ++m) A[k][m] = std::pow(2.0 * m + 1.0, 2.0 * k + 1.0);
        A[k][4] = std::pow(r * r, (double)k) - shift;
    }
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int rr = col + 1; rr < 4; ++rr)
            if (std::fabs(A[rr][col]) > std::fabs(A[piv][col])) piv = rr;
        for (int j = 0; j < 5; ++j) std::swap(A[col][j], A[piv][j]);
        for (int rr = col + 1; rr < 4; ++rr) {
            const double f = A[rr][col] / A[col][col];
            for (int j = col; j < 5; ++j) A[rr][j] -= f * A[col][j];
        }
    }
    for (int m = 3; m >= 0; --m) {
        double acc = A[m][4];
        for (int j = m + 1; j < 4; ++j) acc -= A[m][j] * out[j];
        out[m] = acc / A[m][m];
    }
}

constexpr int64_t kAlignCells = 64;
constexpr int64_t kRowCells = 32;        // row pitch granule of 2D/3D domains: one 128-byte line
constexpr int64_t kAlignBytes = 256;
// 2D grids: tile kernels (64 x plane_rows tiles, LDS halos, one tile per block)
// rather than the marching kernels when the plane-kernel option is auto.
// Measured per step, marching against 8-row tiles: 1.768 / 1.509 ms on 64
// ragged shots of 384^2..1536^2 (N = 4), 0.424 / 0.340 ms on 16 x 1024^2,
// 0.120 / 0.092 ms on 2048^2 (N = 4), 0.102 / 0.068 ms on 2048^2 (N = 2)
constexpr bool kTile2dDefault = true;

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Device buffer owned by the library (small tables only).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release()
    {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n)
    {
        if (n <= bytes && ptr) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&ptr, std::max<size_t>(n, 256));
        if (e == hipSuccess) bytes = std::max<size_t>(n, 256);
        return e;
    }
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

}  // namespace

struct fw_sim {
    // grid
    int ndim = 0, n_domains = 0, nmech = 0, pml = 0;
    double dx = 0, dt = 0;
    double pml_R0 = 1e-4, pml_falpha = 1e6, pml_cref = 0;
    std::vector<fw::DomainDesc> doms;
    int64_t total_cells = 0;
    // workspace layout (byte offsets)
    int64_t off_p = 0, off_v[3] = {0, 0, 0}, off_psi1[3] = {0, 0, 0}, off_psi2 = 0;
    int64_t off_pP1[3] = {0, 0, 0}, off_pP2[3] = {0, 0, 0}, state_end = 0, off_cls = 0, ws_bytes = 0;
    bool have_v[3] = {false, false, false};
    char *ws = nullptr;
    // media
    bool media_set = false, table_set = false;
    int n_classes = 0;
    std::vector<double> c, rho, beta;
    double noise_amp = 0;
    const float *amap = nullptr;         // caller's per-voxel strength scale (fw_set_strength_map), borrowed
    uint64_t noise_seed = 0;
    std::vector<double> kappa, dcoef, alpha;
    std::vector<double> alpha0;          // power-law coefficient per class (fw_set_class_alpha0)
    // staggered first-derivative coefficients (Taylor, or the time-space set of
    // fw_set_time_space_stencil) and the smallest kappa1 kappa2 of the table
    // and the off-axis weight b of the widened 2D stencil (fw_set_widened_stencil)
    double fd[4] = {kFD[0], kFD[1], kFD[2], kFD[3]};
    double fd_b = 0.0, fd_cref = 0.0, min_kk = 1.0;
    // bound of one axis's difference symbol: sum |c_m| + 2 (ndim - 1) |b|
    double fd_abs_sum() const
    {
        return std::fabs(fd[0]) + std::fabs(fd[1]) + std::fabs(fd[2]) + std::fabs(fd[3]) +
               2.0 * (ndim - 1) * std::fabs(fd_b);
    }
    // device tables
    DevBuf d_doms, d_classes, d_pml, d_tiles, d_vtiles, d_ptiles, d_waves, d_traces, d_step;
    float *traces_ext = nullptr;         // caller-owned trace buffer (fw_set_receivers_into), borrowed
    // interleaved 3D schedule (FW_OPT_STEP_CHUNK): per chunk, the velocity
    // tiles of planes [cC, (c+1)C) and the pressure tiles of [cC-3, (c+1)C-3)
    struct ChunkList {
        int64_t voff, poff;
        int32_t vn, vper, pn, pper;
    };
    int step_chunk = -1;                 // -1: automatic (kStepChunk on large grids), 0: off
    std::vector<ChunkList> chunks;
    DevBuf d_vchunks, d_pchunks;
    float *traces() const { return traces_ext ? traces_ext : d_traces.as<float>(); }
    DevBuf d_srcrec, d_rec_of, d_sr_range;
    int64_t n_sr_range = 0;                        // entries uploaded to d_sr_range (n_domains + 1, or 0)
    int resident = -1;                             // resident 1D step: -1 / 1 where it applies, 0 off
    std::vector<int64_t> h_src_cell, h_rec_cell;   // global cells of the sources and the receivers
    std::vector<int32_t> h_src_wave;               // waveform row of each source
    int64_t n_srcrec = 0;
    DevBuf d_cadj, d_adj_cells, d_adj_off, d_adj_idx, d_chain;
    DevBuf d_pold, d_partial, d_check;
    int64_t n_adj_cells = 0;
    int64_t total_packed = 0;
    int n_tiles = 0, tiles_per_xcd = 0, n_vtiles = 0, vtiles_per_xcd = 0, n_ptiles = 0, ptiles_per_xcd = 0;
    std::vector<int32_t> h_tile_dom;     // domain of each marching tile (energy partial sums)
    int64_t n_src = 0, n_rec = 0;
    int n_t = 0, n_t_max = 0;
    // options
    int graph_steps = 16, march_chunk = 0, tile_rows = 4, rows_per_thread = 1, persistent = 0, tile_order = 0,
        plane_kernels = -1, plane_rows = 4, vel_planes = 1, prs_planes = 2;   // per dimension and N: fw_create_grid
    // stepping
    int64_t host_step = 0;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_len = 0;
    bool tiles_dirty = true;

    ~fw_sim()
    {
        drop_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
    void drop_graph()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        graph_exec = nullptr;
        graph_len = 0;
    }
    // cells of domain d, and the cells it occupies in the padded rows
    int64_t cells(int d) const { return doms[d].n[0] * doms[d].n[1] * doms[d].n[2]; }
    int64_t stored(int d) const { return (int64_t)doms[d].pitch * doms[d].n[1] * doms[d].n[2]; }
    // stored position of a domain-local (unpadded) cell index
    int64_t stored_index(int d, int64_t cell) const
    {
        return (cell / doms[d].n[0]) * doms[d].pitch + cell % doms[d].n[0];
    }
};

namespace {

void layout(fw_sim *s)
{
    int64_t off = 0;
    const int64_t fbytes = s->total_cells * 4;
    const int64_t vbytes = s->total_cells * 4 * s->nmech;
    auto take = [&](int64_t bytes) {
        const int64_t o = off;
        off = align_up(off + bytes, kAlignBytes);
        return o;
    };
    s->off_p = take(fbytes);
    for (int a = 0; a < 3; ++a) {
        s->have_v[a] = a < s->ndim;
        s->off_v[a] = take(s->have_v[a] ? fbytes : 0);
    }
    for (int a = 0; a < 3; ++a) s->off_psi1[a] = take(a < s->ndim ? vbytes : 0);
    s->off_psi2 = take(vbytes);
    for (int a = 0; a < 3; ++a) s->off_pP1[a] = take(s->pml > 0 && a < s->ndim ? fbytes : 0);
    for (int a = 0; a < 3; ++a) s->off_pP2[a] = take(s->pml > 0 && a < s->ndim ? fbytes : 0);
    s->state_end = off;
    s->off_cls = take(s->total_cells);
    s->ws_bytes = off;
}

fw::Fields fields_at(const fw_sim *s, char *w)
{
    fw::Fields f{};
    f.p = reinterpret_cast<float *>(w + s->off_p);
    f.vx = reinterpret_cast<float *>(w + s->off_v[0]);
    f.vy = reinterpret_cast<float *>(w + s->off_v[1]);
    f.vz = reinterpret_cast<float *>(w + s->off_v[2]);
    f.psi1x = reinterpret_cast<float *>(w + s->off_psi1[0]);
    f.psi1y = reinterpret_cast<float *>(w + s->off_psi1[1]);
    f.psi1z = reinterpret_cast<float *>(w + s->off_psi1[2]);
    f.psi2 = reinterpret_cast<float *>(w + s->off_psi2);
    for (int a = 0; a < 3; ++a) {
        f.pP1[a] = reinterpret_cast<float *>(w + s->off_pP1[a]);
        f.pP2[a] = reinterpret_cast<float *>(w + s->off_pP2[a]);
    }
    f.cls = reinterpret_cast<uint8_t *>(s->ws + s->off_cls);
    return f;
}

fw::Fields fields_of(const fw_sim *s) { return fields_at(s, s->ws); }

// CPML recursion coefficients along one axis of n points (kappa = 1):
// d = d0 delta^2, alpha = pi f_alpha (1 - delta), b = exp(-(d + alpha) dt),
// a = d / (d + alpha) (b - 1); delta = depth from the slab's inner edge.
void pml_axis(const fw_sim *s, int64_t n, double cref, bool faces, double *a, double *b)
{
    const int P = s->pml;
    const double d0 = P > 0 ? 3.0 * cref * std::log(1.0 / s->pml_R0) / (2.0 * P * s->dx) : 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double x = (double)i + (faces ? 0.5 : 0.0);
        double delta = 0.0;
        if (P > 0) {
            delta = std::max(0.0, std::max((P - 0.5 - x) / P, (x - ((double)n - P - 0.5)) / P));
            delta = std::min(delta, 1.0);
        }
        const double d = d0 * delta * delta;
        const double al = M_PI * s->pml_falpha * (1.0 - delta);
        const double bb = std::exp(-(d + al) * s->dt);
        b[i] = bb;
        a[i] = d > 0.0 ? d / (d + al) * (bb - 1.0) : 0.0;
    }
}

int stability_check(const fw_sim *s, double min_kappa_prod)
{
    double cmax = 0;
    for (double v : s->c) cmax = std::max(cmax, v);
    const double courant = cmax * (1.0 + s->noise_amp) * s->dt / s->dx * std::sqrt((double)s->ndim) * s->fd_abs_sum() /
                           std::sqrt(min_kappa_prod);
    if (!(courant < 1.0))
        return fail(FW_EUNSTABLE, "time step too large: c_max dt/dx sqrt(ndim) sum|c_m| / sqrt(kappa1 kappa2) = %.6f >= 1",
                    courant);
    return FW_OK;
}

// Plane-major tile list in 8 segments, one per XCD: segment k holds y-band k
// (of the y-tiles) of every chunk of planes, domain by domain; segments are
// padded with empty tiles (z1 == z0, skipped by every kernel) to one length.
// Only planes [zlo, zhi) of each domain when given (the interleaved schedule).
static std::vector<fw::Tile> banded_tiles(const fw_sim *s, int tx, int ty, int64_t chunk_or_auto, int64_t zlo = 0,
                                          int64_t zhi = std::numeric_limits<int64_t>::max())
{
    std::vector<fw::Tile> seg[8];
    for (int d = 0; d < s->n_domains; ++d) {
        const int64_t nx = s->doms[d].n[0], ny = s->doms[d].n[1], nz = s->doms[d].n[2];
        const int64_t nytile = (ny + ty - 1) / ty, nxtile = (nx + tx - 1) / tx;
        int64_t chunk = chunk_or_auto;
        if (chunk <= 0) {
            const int64_t nch = (nz + 47) / 48;
            chunk = (nz + nch - 1) / nch;
        }
        chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, nz));
        const int64_t za = std::max<int64_t>(0, zlo), zb = std::min(nz, zhi);
        for (int64_t z0 = za; z0 < zb; z0 += chunk)
            for (int k = 0; k < 8; ++k)
                for (int64_t yt = k * nytile / 8; yt < (k + 1) * nytile / 8; ++yt)
                    for (int64_t xt = 0; xt < nxtile; ++xt) {
                        fw::Tile t{};
                        t.dom = d;
                        t.x0 = (int32_t)(xt * tx);
                        t.y0 = (int32_t)(yt * ty);
                        t.z0 = (int32_t)z0;
                        t.z1 = (int32_t)std::min(zb, z0 + chunk);
                        seg[k].push_back(t);
                    }
    }
    size_t len = 0;
    for (int k = 0; k < 8; ++k) len = std::max(len, seg[k].size());
    std::vector<fw::Tile> tiles;
    tiles.reserve(8 * len);
    for (int k = 0; k < 8; ++k) {
        tiles.insert(tiles.end(), seg[k].begin(), seg[k].end());
        tiles.insert(tiles.end(), len - seg[k].size(), fw::Tile{});
    }
    return tiles;
}

static int upload_tiles(const std::vector<fw::Tile> &tiles, DevBuf &buf, int *n, int *per_xcd)
{
    if (tiles.size() > (size_t)std::numeric_limits<int32_t>::max() - 8)
        return fail(FW_EINVAL, "too many tiles (%zu): use longer march chunks", tiles.size());
    *n = (int)tiles.size();
    *per_xcd = (*n + 7) / 8;
    if (tiles.empty()) return FW_OK;
    HIP_OR_FAIL(buf.ensure(tiles.size() * sizeof(fw::Tile)));
    HIP_OR_FAIL(hipMemcpy(buf.ptr, tiles.data(), tiles.size() * sizeof(fw::Tile), hipMemcpyHostToDevice));
    return FW_OK;
}

// plane kernels in use for the 3D updates (2D: the tile kernels): option 1
// or -1 (default) for both, 0 for neither.  On 960 x 960 x 720 the plane
// kernels take the step from 24.13 to 21.54 ms at N = 4, 20.31 to 18.42 at
// N = 3, 16.65 to 15.06 at N = 2 and 13.70 to 11.71 at N = 1 (marching
// velocity with plane pressure: 12.64)
static bool plane_velocity_on(const fw_sim *s)
{
    if (s->ndim == 2) return s->plane_kernels == 1 || (s->plane_kernels < 0 && kTile2dDefault);
    return s->ndim == 3 && s->plane_kernels != 0;
}

static bool plane_pressure_on(const fw_sim *s)
{
    if (s->ndim == 2) return s->plane_kernels == 1 || (s->plane_kernels < 0 && kTile2dDefault);
    return s->ndim == 3 && s->plane_kernels != 0;
}

// Interleaved schedule: velocity over planes [cC, (c+1)C), then pressure
// over [cC - 3, (c+1)C - 3) (from 0 for the first chunk, to the last plane for
// the last).  The pressure update of plane j reads v_z of planes up to j + 3,
// all updated by then; the velocity update of plane j reads p of planes down
// to j - 3, none of which an earlier pressure chunk has written.  So every
// cell sees the same operands as in the two whole-grid launches (same bits),
// while the planes the pressure update reads again were touched one chunk
// earlier.
// Automatic choice (measured, per graph-replayed step, whole-grid / 120-plane
// chunks): 960 x 960 x 720 N = 4 21.65 / 21.45 ms, 499 x 499 x 1247 N = 2
// 7.41 / 7.27 ms, 512^3 N = 4 4.38 / 4.33 ms; on 256^3 the chunks' extra
// launch tails cost more than they save (0.537 / 0.553 ms with 128 planes),
// so grids of fewer than 480 planes or 200 k cells per plane keep whole-grid
// launches.
constexpr int64_t kStepChunk = 120, kChunkMinPlanes = 320, kChunkMinPlaneCells = 100000;

static int build_chunk_lists(fw_sim *s)
{
    s->chunks.clear();
    if (s->step_chunk == 0 || s->ndim != 3 || !plane_velocity_on(s) || !plane_pressure_on(s)) return FW_OK;
    int64_t nzmax = 0, plane_max = 0;
    for (const auto &d : s->doms) {
        nzmax = std::max<int64_t>(nzmax, d.n[2]);
        plane_max = std::max<int64_t>(plane_max, d.n[0] * d.n[1]);
    }
    if (s->step_chunk < 0 && (nzmax < kChunkMinPlanes || plane_max < kChunkMinPlaneCells)) return FW_OK;
    const int64_t C = s->step_chunk < 0 ? kStepChunk : s->step_chunk;
    const int64_t nch = (nzmax + C - 1) / C;
    std::vector<fw::Tile> va, pa;
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t plo = c == 0 ? 0 : c * C - 3;
        const int64_t phi = c + 1 == nch ? nzmax : (c + 1) * C - 3;
        std::vector<fw::Tile> v = banded_tiles(s, 64, s->plane_rows, s->vel_planes, c * C, (c + 1) * C);
        std::vector<fw::Tile> p = banded_tiles(s, 64, s->plane_rows, s->prs_planes, plo, phi);
        fw_sim::ChunkList L{};
        L.voff = (int64_t)va.size();
        L.vn = (int32_t)v.size();
        L.vper = (L.vn + 7) / 8;
        L.poff = (int64_t)pa.size();
        L.pn = (int32_t)p.size();
        L.pper = (L.pn + 7) / 8;
        va.insert(va.end(), v.begin(), v.end());
        pa.insert(pa.end(), p.begin(), p.end());
        s->chunks.push_back(L);
    }
    if (va.size() > (size_t)std::numeric_limits<int32_t>::max() || pa.size() > (size_t)std::numeric_limits<int32_t>::max())
        return fail(FW_EINVAL, "too many tiles in the interleaved schedule");
    if (!va.empty()) {
        HIP_OR_FAIL(s->d_vchunks.ensure(va.size() * sizeof(fw::Tile)));
        HIP_OR_FAIL(hipMemcpy(s->d_vchunks.ptr, va.data(), va.size() * sizeof(fw::Tile), hipMemcpyHostToDevice));
    }
    if (!pa.empty()) {
        HIP_OR_FAIL(s->d_pchunks.ensure(pa.size() * sizeof(fw::Tile)));
        HIP_OR_FAIL(hipMemcpy(s->d_pchunks.ptr, pa.data(), pa.size() * sizeof(fw::Tile), hipMemcpyHostToDevice));
    }
    return FW_OK;
}

int build_tiles(fw_sim *s)
{
    int tx, ty;
    fw::tile_shape(s->ndim, s->tile_rows, &tx, &ty);
    std::vector<fw::Tile> tiles;
    if (s->tile_order == 2 && s->ndim == 3) {
        tiles = banded_tiles(s, tx, ty, s->march_chunk);
    } else {
        for (int d = 0; d < s->n_domains; ++d) {
            const int64_t nx = s->doms[d].n[0], ny = s->doms[d].n[1], nz = s->doms[d].n[2];
            const int64_t nmarch = s->ndim == 3 ? nz : (s->ndim == 2 ? ny : 1);
            const int64_t nytile = s->ndim == 3 ? (ny + ty - 1) / ty : 1;
            const int64_t nxtile = (nx + tx - 1) / tx;
            int64_t chunk = s->march_chunk;
            if (chunk <= 0 && s->ndim == 3) {
                // about 48 planes per tile (measured best: many small 4-wave tiles
                // keep several independent blocks on each CU)
                const int64_t nch = (nmarch + 47) / 48;
                chunk = (nmarch + nch - 1) / nch;
            } else if (chunk <= 0) {
                // 2D: 8 rows per one-wave tile (measured best on single and
                // batched grids: the many short tiles keep more waves in flight
                // than the queue warm-up of each tile costs); 1D: one row
                chunk = 8;
            }
            chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, nmarch));
            // tile order inside a chunk: x fastest (order 0) or y fastest
            // (order 1: the y neighbours of a tile run right after it, so the
            // halo rows they share are still in L2 when the second one reads them)
            const int64_t n_in = nxtile * nytile;
            for (int64_t z0 = 0; z0 < nmarch; z0 += chunk)
                for (int64_t k = 0; k < n_in; ++k) {
                    const int64_t xt = s->tile_order == 1 ? k / nytile : k % nxtile;
                    const int64_t yt = s->tile_order == 1 ? k % nytile : k / nxtile;
                    fw::Tile t{};
                    t.dom = d;
                    t.x0 = (int32_t)(xt * tx);
                    t.y0 = (int32_t)(yt * ty);
                    t.z0 = (int32_t)z0;
                    t.z1 = (int32_t)std::min(nmarch, z0 + chunk);
                    tiles.push_back(t);
                }
        }
    }
    int rc = upload_tiles(tiles, s->d_tiles, &s->n_tiles, &s->tiles_per_xcd);
    if (rc != FW_OK) return rc;
    s->h_tile_dom.resize(tiles.size());
    for (size_t t = 0; t < tiles.size(); ++t) s->h_tile_dom[t] = tiles[t].dom;
    // plane-kernel tiles (3D; 2D tile kernels): 64 x plane_rows, vel_planes planes
    // each for the velocity update, prs_planes for the pressure update (2D: one)
    std::vector<fw::Tile> vt, pt;
    if (plane_velocity_on(s)) vt = banded_tiles(s, 64, s->plane_rows, s->vel_planes);
    if (plane_pressure_on(s)) pt = banded_tiles(s, 64, s->plane_rows, s->prs_planes);
    rc = upload_tiles(vt, s->d_vtiles, &s->n_vtiles, &s->vtiles_per_xcd);
    if (rc != FW_OK) return rc;
    rc = upload_tiles(pt, s->d_ptiles, &s->n_ptiles, &s->ptiles_per_xcd);
    if (rc != FW_OK) return rc;
    rc = build_chunk_lists(s);
    if (rc != FW_OK) return rc;
    s->tiles_dirty = false;
    s->drop_graph();
    return FW_OK;
}

fw::StepArgs step_args(const fw_sim *s)
{
    fw::StepArgs a{};
    a.f = fields_of(s);
    a.fo = a.f;
    a.doms = s->d_doms.as<fw::DomainDesc>();
    a.tiles = s->d_tiles.as<fw::Tile>();
    a.classes = s->d_classes.as<fw::ClassCoef>();
    a.pml_tab = s->d_pml.as<float>();
    a.n_tiles = s->n_tiles;
    a.tiles_per_xcd = s->tiles_per_xcd;
    a.blocks_per_xcd = s->persistent > 0 ? std::max(1, std::min(s->tiles_per_xcd, s->persistent * 32))
                                         : s->tiles_per_xcd;
    a.pml = s->pml;
    int cap = 1;
    for (const auto &d : s->doms) cap = std::max(cap, (int)d.n_classes);
    a.class_cap = (cap + 3) / 4 * 4;
    a.tile_rows = s->tile_rows;
    // the plane kernels take one tile per block: not with a persistent grid
    a.plane = (plane_velocity_on(s) && s->persistent == 0 && s->n_vtiles > 0) ? 1 : 0;
    a.plane_p = (plane_pressure_on(s) && s->persistent == 0 && s->n_ptiles > 0) ? 1 : 0;
    a.plane_rows = s->plane_rows;
    a.vel_planes = s->vel_planes;
    a.prs_planes = s->prs_planes;
    a.vtiles = s->d_vtiles.as<fw::Tile>();
    a.n_vtiles = s->n_vtiles;
    a.vtiles_per_xcd = s->vtiles_per_xcd;
    a.ptiles = s->d_ptiles.as<fw::Tile>();
    a.n_ptiles = s->n_ptiles;
    a.ptiles_per_xcd = s->ptiles_per_xcd;
    for (int m = 0; m < 4; ++m) a.fd[m] = (float)(s->fd[m] / s->dx);
    a.fd_b = (float)(s->fd_b / s->dx);
    a.dt = (float)s->dt;
    a.noise_amp = (float)s->noise_amp;
    a.amap = s->amap;
    return a;
}

fw::SrcRecArgs srcrec_args(const fw_sim *s)
{
    fw::SrcRecArgs a{};
    a.p = fields_of(s).p;
    a.cells = s->d_srcrec.as<fw::SrcRecCell>();
    a.n_cells = s->n_srcrec;
    a.rec_of = s->d_rec_of.as<int32_t>();
    a.waves = s->d_waves.as<float>();
    a.n_t = s->n_t;
    a.traces = s->traces();
    a.n_rec = s->n_rec;
    a.n_t_max = s->n_t_max;
    a.step = s->d_step.as<int64_t>();
    a.bad_row = s->d_step.as<int64_t>() + 1;
    a.done = reinterpret_cast<uint32_t *>(s->d_step.as<int64_t>() + 2);
    return a;
}

// The resident 1D step applies to 1D grids whose domains all fit on chip,
// with CPML slabs of at most kResident1dSlab cells together and no strength
// map (the per-step kernels take the map).
static bool resident_on(const fw_sim *s)
{
    if (s->resident == 0 || s->ndim != 1 || s->amap || 2 * s->pml > fw::kResident1dSlab) return false;
    for (const auto &d : s->doms)
        if (d.n[0] > fw::kResident1dCells) return false;
    return true;
}

// n steps of the resident 1D kernel, in launches of at most kResidentSteps
// steps (a launch holds its domains' workgroups for its whole run).
constexpr int kResidentSteps = 4096;
static int enqueue_resident(fw_sim *s, int n, hipStream_t st)
{
    const fw::SrcRecArgs r = srcrec_args(s);
    fw::Resident1dArgs a{};
    a.s = step_args(s);
    a.cells = r.cells;
    // no source or receiver set yet: no ranges (the kernel then has none)
    a.sr_range = s->n_sr_range == s->n_domains + 1 ? s->d_sr_range.as<int32_t>() : nullptr;
    a.rec_of = r.rec_of;
    a.waves = r.waves;
    a.n_t = r.n_t;
    a.traces = r.traces;
    a.n_rec = r.n_rec;
    a.n_t_max = r.n_t_max;
    a.step = r.step;
    a.bad_row = r.bad_row;
    a.done = r.done;
    for (int left = n; left > 0;) {
        a.n_steps = std::min(left, kResidentSteps);
        HIP_OR_FAIL(fw::launch_resident1d(s->nmech, a, s->n_domains, st));
        left -= a.n_steps;
    }
    return FW_OK;
}

// The step's arguments restricted to one chunk of the interleaved schedule.
static fw::StepArgs chunk_args(const fw_sim *s, const fw::StepArgs &a, const fw_sim::ChunkList &L)
{
    fw::StepArgs c = a;
    c.vtiles = s->d_vchunks.as<fw::Tile>() + L.voff;
    c.n_vtiles = L.vn;
    c.vtiles_per_xcd = L.vper;
    c.ptiles = s->d_pchunks.as<fw::Tile>() + L.poff;
    c.n_ptiles = L.pn;
    c.ptiles_per_xcd = L.pper;
    return c;
}

static bool interleaved_on(const fw_sim *s, const fw::StepArgs &a)
{
    return !s->chunks.empty() && a.plane && a.plane_p;
}

int enqueue_steps(fw_sim *s, int n, hipStream_t st)
{
    const fw::StepArgs a = step_args(s);
    if (s->fd_b != 0.0 && !(a.plane && a.plane_p))
        return fail(FW_EUNSUPPORTED, "the widened stencil runs on the 2D tile kernels only (FW_OPT_PLANE_KERNELS "
                                     "off or a persistent grid selected)");
    const fw::SrcRecArgs r = srcrec_args(s);
    const bool interleaved = interleaved_on(s, a);
    for (int i = 0; i < n; ++i) {
        if (interleaved) {
            for (const auto &L : s->chunks) {
                const fw::StepArgs c = chunk_args(s, a, L);
                if (L.vn > 0)
                    HIP_OR_FAIL(fw::launch_velocity(s->ndim, s->nmech, s->tile_rows, s->rows_per_thread, c, st));
                if (L.pn > 0)
                    HIP_OR_FAIL(fw::launch_pressure(s->ndim, s->nmech, s->tile_rows, s->rows_per_thread, c, st));
            }
        } else {
            HIP_OR_FAIL(fw::launch_velocity(s->ndim, s->nmech, s->tile_rows, s->rows_per_thread, a, st));
            HIP_OR_FAIL(fw::launch_pressure(s->ndim, s->nmech, s->tile_rows, s->rows_per_thread, a, st));
        }
        HIP_OR_FAIL(fw::launch_src_rec(r, st));
    }
    return FW_OK;
}

int ensure_graph(fw_sim *s, int len)
{
    if (s->graph_exec && s->graph_len == len) return FW_OK;
    s->drop_graph();
    if (!s->cap_stream) HIP_OR_FAIL(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    HIP_OR_FAIL(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_steps(s, len, s->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
    if (rc != FW_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(FW_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(FW_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    s->graph_exec = ex;
    s->graph_len = len;
    return FW_OK;
}

bool check_ptr(const void *p) { return p != nullptr; }

}  // namespace

extern "C" {

const char *fw_last_error(void) { return g_err.c_str(); }

int fw_abi_version(void) { return 2; }

int fw_create_grid(fw_sim **out, int ndim, int n_domains, const int64_t *shape, double dx, double dt, int n_mech,
                   int pml_cells, const double *pml_params)
{
    g_err.clear();
    if (!out) return fail(FW_EINVAL, "out is NULL");
    *out = nullptr;
    if (ndim < 1 || ndim > 3) return fail(FW_EINVAL, "ndim must be 1, 2 or 3 (got %d)", ndim);
    if (n_domains < 1) return fail(FW_EINVAL, "n_domains must be >= 1 (got %d)", n_domains);
    if (!shape) return fail(FW_EINVAL, "shape is NULL");
    if (!(dx > 0) || !(dt > 0) || !std::isfinite(dx) || !std::isfinite(dt))
        return fail(FW_EINVAL, "dx and dt must be finite and > 0");
    if (n_mech < 1 || n_mech > fw::kMaxMech) return fail(FW_EINVAL, "n_mech must be in 1..4 (got %d)", n_mech);
    if (pml_cells < 0) return fail(FW_EINVAL, "pml_cells must be >= 0");
    fw_sim *s = new (std::nothrow) fw_sim();
    if (!s) return fail(FW_ENOMEM, "out of host memory");
    s->ndim = ndim;
    s->n_domains = n_domains;
    s->nmech = n_mech;
    // pressure plane-kernel tile depth by mechanism count (measured on
    // 960 x 960 x 720: N = 4, 6.77 / 6.97 / 7.05 ms with 2 / 4 / 8 planes, the
    // 2-plane kernel fitting 8 waves per SIMD; N = 2, 5.54 / 5.78 / 5.65 ms
    // and 3.13 / 3.14 / 3.17 ms on 499 x 499 x 1247 with 8 / 4 / 2)
    s->prs_planes = n_mech >= 3 ? 2 : 8;
    // 2D tile kernels: 8-row tiles (measured against 4 / 16 rows: 0.340 /
    // 0.351 / 0.343 ms per step on 16 shots of 1024^2 at N = 4, 0.068 / 0.071 /
    // 0.072 ms on 2048^2 at N = 2, equal on the 64-shot ragged batch)
    if (ndim == 2) s->plane_rows = 8;
    // 3D plane kernels at N <= 2: 8-row tiles, two planes per velocity tile
    // (measured, step ms with rows 4 / 8 and 1 / 2 / 4 velocity planes:
    // 960 x 960 x 720 15.83 15.76 15.94 / 16.02 15.56 15.71; 499 x 499 x 1247
    // 8.13 7.97 7.88 / 7.93 7.69 7.60; at N = 4 the 4-row, 1-plane default is
    // fastest: 21.79 against 22.05-23.44)
    if (ndim == 3 && n_mech <= 2) {
        s->plane_rows = 8;
        s->vel_planes = 2;
    }
    s->pml = pml_cells;
    s->dx = dx;
    s->dt = dt;
    if (pml_params) {
        s->pml_R0 = pml_params[0];
        s->pml_falpha = pml_params[1];
        s->pml_cref = pml_params[2];
        if (!(s->pml_R0 > 0 && s->pml_R0 < 1) || !(s->pml_falpha >= 0) || !(s->pml_cref >= 0)) {
            delete s;
            return fail(FW_EINVAL, "pml_params: need 0 < R0 < 1, f_alpha >= 0, c_ref >= 0");
        }
    }
    int64_t off = 0;
    for (int d = 0; d < n_domains; ++d) {
        fw::DomainDesc D{};
        for (int a = 0; a < 3; ++a) {
            const int64_t n = shape[3 * d + a];
            if (a < ndim) {
                if (n <= 2 * (int64_t)pml_cells + 8 || n > (int64_t)INT32_MAX) {
                    delete s;
                    return fail(FW_EINVAL, "domain %d axis %d: size %lld must exceed 2*pml_cells+8 = %d", d, a,
                                (long long)n, 2 * pml_cells + 8);
                }
            } else if (n != 1) {
                delete s;
                return fail(FW_EINVAL, "domain %d axis %d: unused dimension must be 1 (got %lld)", d, a, (long long)n);
            }
            D.n[a] = n;
        }
        // rows padded to whole 128-byte lines in 2D and 3D: a row of a 64-cell
        // tile then spans two lines, not three (measured on 961 x 960 x 720 at
        // N = 4: 29.1 ms per step unpadded against 21.8 ms for 960 wide)
        D.pitch = (int32_t)(ndim >= 2 ? align_up(D.n[0], kRowCells) : D.n[0]);
        D.cell_off = off;
        D.packed_off = s->total_packed;
        if ((int64_t)D.pitch * D.n[1] * D.n[2] >= ((int64_t)1 << 31)) {
            delete s;
            return fail(FW_EINVAL, "domain %d has 2^31 cells or more (rows padded to %d cells)", d, (int)kRowCells);
        }
        off = align_up(off + (int64_t)D.pitch * D.n[1] * D.n[2], kAlignCells);
        s->total_packed += D.n[0] * D.n[1] * D.n[2];
        s->doms.push_back(D);
    }
    s->total_cells = off;
    layout(s);
    *out = s;
    return FW_OK;
}

int fw_destroy(fw_sim *sim)
{
    delete sim;
    return FW_OK;
}

int64_t fw_workspace_bytes(const fw_sim *sim) { return sim ? sim->ws_bytes : -1; }

int fw_bind_workspace(fw_sim *sim, void *d_ptr, int64_t bytes)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (!d_ptr) return fail(FW_EINVAL, "workspace pointer is NULL");
    if ((reinterpret_cast<uintptr_t>(d_ptr) % kAlignBytes) != 0) return fail(FW_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < sim->ws_bytes)
        return fail(FW_ENOMEM, "workspace too small: %lld < %lld bytes", (long long)bytes, (long long)sim->ws_bytes);
    sim->ws = static_cast<char *>(d_ptr);
    HIP_OR_FAIL(hipMemset(sim->ws, 0, (size_t)sim->ws_bytes));
    // [0] step counter, [1] first trace row with a non-finite value (-1)
    // step counter, first non-finite trace row (-1), workgroups finished in
    // the running source/receiver launch (0)
    HIP_OR_FAIL(sim->d_step.ensure(3 * sizeof(int64_t)));
    HIP_OR_FAIL(hipMemset(sim->d_step.ptr, 0, 3 * sizeof(int64_t)));
    HIP_OR_FAIL(hipMemset(static_cast<char *>(sim->d_step.ptr) + sizeof(int64_t), 0xff, sizeof(int64_t)));
    sim->host_step = 0;
    sim->media_set = sim->table_set = false;
    sim->drop_graph();
    return FW_OK;
}

int fw_set_media(fw_sim *sim, const uint8_t *h_class, const int32_t *class_base, int n_classes, const double *c,
                 const double *rho, const double *beta, double c_noise_amp, uint64_t noise_seed)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (!check_ptr(h_class) || !check_ptr(class_base) || !check_ptr(c) || !check_ptr(rho) || !check_ptr(beta))
        return fail(FW_EINVAL, "NULL array argument");
    if (n_classes < 1) return fail(FW_EINVAL, "n_classes must be >= 1");
    if (!(c_noise_amp >= 0 && c_noise_amp < 0.5)) return fail(FW_EINVAL, "c_noise_amp must be in [0, 0.5)");
    for (int k = 0; k < n_classes; ++k) {
        if (!(c[k] > 0) || !(rho[k] > 0) || !std::isfinite(c[k]) || !std::isfinite(rho[k]))
            return fail(FW_EINVAL, "class %d: c and rho must be finite and > 0", k);
        if (!std::isfinite(beta[k])) return fail(FW_EINVAL, "class %d: beta must be finite", k);
    }
    // class indices: local < 256 (uint8) and base + local < n_classes
    int64_t pos = 0;
    std::vector<int> ncls(sim->n_domains, 0);
    for (int d = 0; d < sim->n_domains; ++d) {
        const int32_t b = class_base[d];
        if (b < 0 || b >= n_classes) return fail(FW_EINVAL, "domain %d: class_base %d out of range", d, b);
        const int64_t nc = sim->cells(d);
        int mx = 0;
        for (int64_t i = 0; i < nc; ++i) mx = std::max<int>(mx, h_class[pos + i]);
        if (b + mx >= n_classes)
            return fail(FW_EINVAL, "domain %d: class index %d + base %d >= n_classes %d", d, mx, b, n_classes);
        ncls[d] = mx + 1;
        pos += nc;
    }
    sim->c.assign(c, c + n_classes);
    sim->rho.assign(rho, rho + n_classes);
    sim->beta.assign(beta, beta + n_classes);
    sim->n_classes = n_classes;
    sim->noise_amp = c_noise_amp;
    sim->noise_seed = noise_seed;
    int rc = stability_check(sim, 1.0);
    if (rc != FW_OK) return rc;
    if (!sim->ws) return fail(FW_ESTATE, "fw_bind_workspace must come first");
    // upload the map
    pos = 0;
    char *dcls = sim->ws + sim->off_cls;
    for (int d = 0; d < sim->n_domains; ++d) {
        const int64_t nc = sim->cells(d);
        const fw::DomainDesc &D = sim->doms[d];
        // rows of nx cells into rows D.pitch apart (the padding keeps class 0)
        HIP_OR_FAIL(hipMemcpy2D(dcls + D.cell_off, (size_t)D.pitch, h_class + pos, (size_t)D.n[0], (size_t)D.n[0],
                                (size_t)(D.n[1] * D.n[2]), hipMemcpyHostToDevice));
        pos += nc;
        sim->doms[d].class_base = class_base[d];
        sim->doms[d].n_classes = ncls[d];
        sim->doms[d].noise_seed = noise_seed;
    }
    // CPML profiles, per domain and axis: [aF | bF | aC | bC] x n
    double cref = sim->pml_cref;
    if (cref <= 0) {
        for (double v : sim->c) cref = std::max(cref, v);
    }
    std::vector<float> tab;
    std::vector<double> a, b;
    for (int d = 0; d < sim->n_domains; ++d) {
        for (int ax = 0; ax < 3; ++ax) {
            const int64_t n = sim->doms[d].n[ax];
            sim->doms[d].pml_off[ax] = (int32_t)tab.size();
            if (ax >= sim->ndim) continue;
            a.resize(n);
            b.resize(n);
            for (int stag = 0; stag < 2; ++stag) {
                pml_axis(sim, n, cref, stag == 0, a.data(), b.data());
                for (int64_t i = 0; i < n; ++i) tab.push_back((float)a[i]);
                for (int64_t i = 0; i < n; ++i) tab.push_back((float)b[i]);
            }
        }
    }
    if (tab.size() > (size_t)INT32_MAX) return fail(FW_EINVAL, "CPML tables too large");
    HIP_OR_FAIL(sim->d_pml.ensure(std::max<size_t>(tab.size(), 1) * sizeof(float)));
    if (!tab.empty()) HIP_OR_FAIL(hipMemcpy(sim->d_pml.ptr, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_OR_FAIL(sim->d_doms.ensure(sim->doms.size() * sizeof(fw::DomainDesc)));
    HIP_OR_FAIL(hipMemcpy(sim->d_doms.ptr, sim->doms.data(), sim->doms.size() * sizeof(fw::DomainDesc),
                          hipMemcpyHostToDevice));
    sim->media_set = true;
    sim->table_set = false;
    sim->tiles_dirty = true;
    sim->drop_graph();
    return FW_OK;
}

int fw_set_relaxation_table(fw_sim *sim, int n_classes, const double *kappa, const double *d, const double *alpha)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (!sim->media_set) return fail(FW_ESTATE, "fw_set_media must come first");
    if (n_classes != sim->n_classes)
        return fail(FW_EINVAL, "n_classes %d differs from fw_set_media (%d)", n_classes, sim->n_classes);
    if (!kappa || !d || !alpha) return fail(FW_EINVAL, "NULL array argument");
    const int N = sim->nmech;
    double min_kk = 1e300;
    std::vector<fw::ClassCoef> cc(n_classes);
    std::vector<fw::ClassAdj> ca(n_classes);
    for (int k = 0; k < n_classes; ++k) {
        fw::ClassCoef &o = cc[k];
        std::memset(&o, 0, sizeof o);
        std::memset(&ca[k], 0, sizeof ca[k]);
        const double k1 = kappa[2 * k], k2 = kappa[2 * k + 1];
        if (!(k1 > 0) || !(k2 > 0) || !std::isfinite(k1) || !std::isfinite(k2))
            return fail(FW_EINVAL, "class %d: kappa must be finite and > 0", k);
        min_kk = std::min(min_kk, k1 * k2);
        o.ik1 = (float)(1.0 / k1);
        o.ik2 = (float)(1.0 / k2);
        o.rho = (float)sim->rho[k];
        o.K = (float)(sim->rho[k] * sim->c[k] * sim->c[k]);
        o.twobeta = (float)(2.0 * sim->beta[k]);
        for (int i = 0; i < 2; ++i) {
            const double kap = i == 0 ? k1 : k2;
            for (int nu = 0; nu < N; ++nu) {
                const double dd = d[(k * 2 + i) * N + nu], al = alpha[(k * 2 + i) * N + nu];
                if (!(dd >= 0) || !(al >= 0) || !std::isfinite(dd) || !std::isfinite(al) || !(dd + kap * al > 0))
                    return fail(FW_EINVAL, "class %d operator %d mechanism %d: need d >= 0, alpha >= 0, d + kappa alpha > 0",
                                k, i + 1, nu);
                // Eqs. (relaxation_b) and (relaxation_a), FP64
                const double bb = std::exp(-(dd / kap + al) * sim->dt);
                const double aa = dd / (kap * (dd + kap * al)) * (bb - 1.0);
                (i == 0 ? o.a1 : o.a2)[nu] = (float)aa;
                (i == 0 ? o.b1 : o.b2)[nu] = (float)bb;
                // derivatives with respect to a scale s of d (d -> s d) at s = 1
                const double bs = -(dd / kap) * sim->dt * bb;
                const double as = dd * al / ((dd + kap * al) * (dd + kap * al)) * (bb - 1.0) +
                                  dd / (kap * (dd + kap * al)) * bs;
                (i == 0 ? ca[k].a1s : ca[k].a2s)[nu] = (float)as;
                (i == 0 ? ca[k].b1s : ca[k].b2s)[nu] = (float)bs;
            }
        }
    }
    int rc = stability_check(sim, min_kk);
    if (rc != FW_OK) return rc;
    sim->min_kk = min_kk;
    sim->kappa.assign(kappa, kappa + 2 * n_classes);
    sim->dcoef.assign(d, d + 2 * N * n_classes);
    sim->alpha.assign(alpha, alpha + 2 * N * n_classes);
    HIP_OR_FAIL(sim->d_classes.ensure(cc.size() * sizeof(fw::ClassCoef)));
    HIP_OR_FAIL(hipMemcpy(sim->d_classes.ptr, cc.data(), cc.size() * sizeof(fw::ClassCoef), hipMemcpyHostToDevice));
    HIP_OR_FAIL(sim->d_cadj.ensure(ca.size() * sizeof(fw::ClassAdj)));
    HIP_OR_FAIL(hipMemcpy(sim->d_cadj.ptr, ca.data(), ca.size() * sizeof(fw::ClassAdj), hipMemcpyHostToDevice));
    sim->table_set = true;
    sim->drop_graph();
    return FW_OK;
}

static int check_cells(const fw_sim *sim, int64_t n, const int32_t *domain, const int64_t *cell,
                       std::vector<int64_t> &global, const char *what)
{
    global.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t d = domain[i];
        if (d < 0 || d >= sim->n_domains) return fail(FW_EINVAL, "%s %lld: domain %d out of range", what, (long long)i, d);
        if (cell[i] < 0 || cell[i] >= sim->cells(d))
            return fail(FW_EINVAL, "%s %lld: cell %lld outside domain %d", what, (long long)i, (long long)cell[i], d);
        global[i] = sim->doms[d].cell_off + sim->stored_index(d, cell[i]);
    }
    return FW_OK;
}

// distinct source/receiver cells (sorted), each with its source and the range
// of its receivers in a list grouped by cell (receivers in index order)
static int build_srcrec(fw_sim *sim)
{
    std::vector<int64_t> cells(sim->h_src_cell);
    cells.insert(cells.end(), sim->h_rec_cell.begin(), sim->h_rec_cell.end());
    std::sort(cells.begin(), cells.end());
    cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
    std::vector<fw::SrcRecCell> tab(cells.size());
    for (size_t e = 0; e < cells.size(); ++e) {
        tab[e] = fw::SrcRecCell{};
        tab[e].cell = cells[e];
        tab[e].wave = -1;
    }
    auto slot = [&](int64_t c) { return (size_t)(std::lower_bound(cells.begin(), cells.end(), c) - cells.begin()); };
    for (size_t i = 0; i < sim->h_src_cell.size(); ++i) tab[slot(sim->h_src_cell[i])].wave = sim->h_src_wave[i];
    const int64_t n_rec = (int64_t)sim->h_rec_cell.size();
    std::vector<int32_t> order(n_rec);
    for (int64_t i = 0; i < n_rec; ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return sim->h_rec_cell[a] < sim->h_rec_cell[b]; });
    for (int64_t k = 0; k < n_rec;) {
        const int64_t c = sim->h_rec_cell[order[k]];
        int64_t k1 = k;
        while (k1 < n_rec && sim->h_rec_cell[order[k1]] == c) ++k1;
        fw::SrcRecCell &e = tab[slot(c)];
        e.r0 = (int32_t)k;
        e.r1 = (int32_t)k1;
        k = k1;
    }
    sim->n_srcrec = (int64_t)tab.size();
    // per domain, its entries of the cell list (the list is sorted and the
    // domains occupy consecutive cell ranges): the resident 1D step's share
    std::vector<int32_t> range((size_t)sim->n_domains + 1, 0);
    for (int d = 0; d <= sim->n_domains; ++d) {
        const int64_t first = d < sim->n_domains ? sim->doms[d].cell_off : std::numeric_limits<int64_t>::max();
        range[d] = (int32_t)(std::lower_bound(cells.begin(), cells.end(), first) - cells.begin());
    }
    HIP_OR_FAIL(sim->d_sr_range.ensure(range.size() * sizeof(int32_t)));
    HIP_OR_FAIL(hipMemcpy(sim->d_sr_range.ptr, range.data(), range.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    sim->n_sr_range = (int64_t)range.size();
    if (!tab.empty()) {
        HIP_OR_FAIL(sim->d_srcrec.ensure(tab.size() * sizeof(fw::SrcRecCell)));
        HIP_OR_FAIL(hipMemcpy(sim->d_srcrec.ptr, tab.data(), tab.size() * sizeof(fw::SrcRecCell), hipMemcpyHostToDevice));
    }
    if (n_rec > 0) {
        HIP_OR_FAIL(sim->d_rec_of.ensure(order.size() * sizeof(int32_t)));
        HIP_OR_FAIL(hipMemcpy(sim->d_rec_of.ptr, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    return FW_OK;
}

int fw_set_sources(fw_sim *sim, int64_t n_src, const int32_t *domain, const int64_t *cell, const int32_t *wave_idx,
                   int n_wave, const float *waves, int n_t)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (n_src < 0) return fail(FW_EINVAL, "n_src must be >= 0");
    if (n_src > 0) {
        if (!domain || !cell || !wave_idx || !waves) return fail(FW_EINVAL, "NULL array argument");
        if (n_wave < 1 || n_t < 1) return fail(FW_EINVAL, "n_wave and n_t must be >= 1");
    }
    std::vector<int64_t> g;
    int rc = check_cells(sim, n_src, domain, cell, g, "source");
    if (rc != FW_OK) return rc;
    for (int64_t i = 0; i < n_src; ++i)
        if (wave_idx[i] < 0 || wave_idx[i] >= n_wave)
            return fail(FW_EINVAL, "source %lld: wave index %d out of range", (long long)i, wave_idx[i]);
    {
        std::vector<int64_t> sorted(g);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(FW_EINVAL, "a source cell appears more than once");
    }
    for (int64_t i = 0; i < (int64_t)n_wave * (n_src > 0 ? n_t : 0); ++i)
        if (!std::isfinite(waves[i])) return fail(FW_ENONFINITE, "source waveform sample %lld is not finite", (long long)i);
    if (!sim->ws) return fail(FW_ESTATE, "fw_bind_workspace must come first");
    sim->n_src = n_src;
    sim->n_t = n_src > 0 ? n_t : 0;
    if (n_src > 0) {
        HIP_OR_FAIL(sim->d_waves.ensure((size_t)n_wave * n_t * sizeof(float)));
        HIP_OR_FAIL(hipMemcpy(sim->d_waves.ptr, waves, (size_t)n_wave * n_t * sizeof(float), hipMemcpyHostToDevice));
    }
    sim->h_src_cell = g;
    sim->h_src_wave.assign(wave_idx, wave_idx + n_src);
    rc = build_srcrec(sim);
    if (rc != FW_OK) return rc;
    sim->drop_graph();
    return FW_OK;
}

// Receivers recording into the library's trace buffer (ext == NULL) or into
// the caller's (ext, cap floats).
static int set_receivers_impl(fw_sim *sim, int64_t n_rec, const int32_t *domain, const int64_t *cell, int n_t_max,
                              float *ext, int64_t cap, bool caller_buffer)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (n_rec < 0 || n_t_max < 0) return fail(FW_EINVAL, "n_rec and n_t_max must be >= 0");
    if (n_rec > 0 && (!domain || !cell)) return fail(FW_EINVAL, "NULL array argument");
    const int64_t need = n_rec > 0 ? n_rec * std::max<int64_t>(n_t_max, 1) : 0;
    if (caller_buffer && n_rec > 0 && !ext) return fail(FW_EINVAL, "d_traces is NULL");
    if (caller_buffer && cap < need)
        return fail(FW_EINVAL, "trace buffer holds %lld floats, %lld needed", (long long)cap, (long long)need);
    std::vector<int64_t> g;
    int rc = check_cells(sim, n_rec, domain, cell, g, "receiver");
    if (rc != FW_OK) return rc;
    if (!sim->ws) return fail(FW_ESTATE, "fw_bind_workspace must come first");
    sim->n_rec = n_rec;
    sim->n_t_max = n_rec > 0 ? n_t_max : 0;
    sim->traces_ext = caller_buffer ? ext : nullptr;
    if (n_rec > 0) {
        const size_t tb = (size_t)need * sizeof(float);
        if (!caller_buffer) HIP_OR_FAIL(sim->d_traces.ensure(tb));
        HIP_OR_FAIL(hipMemset(sim->traces(), 0, tb));
        // receivers grouped by distinct cell, for the adjoint source injection
        std::vector<int32_t> order(n_rec);
        for (int64_t i = 0; i < n_rec; ++i) order[i] = (int32_t)i;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return g[a] < g[b]; });
        std::vector<int64_t> cells;
        std::vector<int32_t> offs;
        for (int64_t k = 0; k < n_rec; ++k) {
            if (k == 0 || g[order[k]] != g[order[k - 1]]) {
                cells.push_back(g[order[k]]);
                offs.push_back((int32_t)k);
            }
        }
        offs.push_back((int32_t)n_rec);
        sim->n_adj_cells = (int64_t)cells.size();
        HIP_OR_FAIL(sim->d_adj_cells.ensure(cells.size() * sizeof(int64_t)));
        HIP_OR_FAIL(sim->d_adj_off.ensure(offs.size() * sizeof(int32_t)));
        HIP_OR_FAIL(sim->d_adj_idx.ensure(order.size() * sizeof(int32_t)));
        HIP_OR_FAIL(hipMemcpy(sim->d_adj_cells.ptr, cells.data(), cells.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        HIP_OR_FAIL(hipMemcpy(sim->d_adj_off.ptr, offs.data(), offs.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_OR_FAIL(hipMemcpy(sim->d_adj_idx.ptr, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    } else {
        sim->n_adj_cells = 0;
    }
    sim->h_rec_cell = g;
    rc = build_srcrec(sim);
    if (rc != FW_OK) return rc;
    sim->drop_graph();
    return FW_OK;
}

int fw_set_receivers(fw_sim *sim, int64_t n_rec, const int32_t *domain, const int64_t *cell, int n_t_max)
{
    return set_receivers_impl(sim, n_rec, domain, cell, n_t_max, nullptr, 0, false);
}

int fw_set_receivers_into(fw_sim *sim, int64_t n_rec, const int32_t *domain, const int64_t *cell, int n_t_max,
                          float *d_traces, int64_t capacity)
{
    return set_receivers_impl(sim, n_rec, domain, cell, n_t_max, d_traces, capacity, true);
}

int fw_prepare(fw_sim *sim)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (!sim->ws || !sim->media_set || !sim->table_set)
        return fail(FW_ESTATE, "bind the workspace, then set media and the relaxation table before preparing");
    if (sim->tiles_dirty) {
        int rc = build_tiles(sim);
        if (rc != FW_OK) return rc;
    }
    return sim->graph_steps > 0 && !resident_on(sim) ? ensure_graph(sim, sim->graph_steps) : FW_OK;
}

int fw_step(fw_sim *sim, int n_steps, void *hip_stream)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (n_steps < 0) return fail(FW_EINVAL, "n_steps must be >= 0");
    if (!sim->ws || !sim->media_set || !sim->table_set)
        return fail(FW_ESTATE, "bind the workspace, then set media and the relaxation table before stepping");
    if (n_steps == 0) return FW_OK;
    if (sim->tiles_dirty) {
        int rc = build_tiles(sim);
        if (rc != FW_OK) return rc;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (resident_on(sim)) {
        int rc = enqueue_resident(sim, n_steps, st);
        if (rc != FW_OK) return rc;
        sim->host_step += n_steps;
        return FW_OK;
    }
    int left = n_steps;
    if (sim->graph_steps > 0 && left >= sim->graph_steps) {
        int rc = ensure_graph(sim, sim->graph_steps);
        if (rc != FW_OK) return rc;
        while (left >= sim->graph_steps) {
            HIP_OR_FAIL(hipGraphLaunch(sim->graph_exec, st));
            left -= sim->graph_steps;
        }
    }
    int rc = enqueue_steps(sim, left, st);
    if (rc != FW_OK) return rc;
    sim->host_step += n_steps;
    return FW_OK;
}

int fw_read_receivers(fw_sim *sim, float *dst, int64_t n_elems, int dst_is_device, void *hip_stream)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (!dst) return fail(FW_EINVAL, "dst is NULL");
    if (n_elems < 0 || n_elems > sim->n_rec * (int64_t)sim->n_t_max)
        return fail(FW_EINVAL, "n_elems %lld exceeds the trace buffer (%lld)", (long long)n_elems,
                    (long long)(sim->n_rec * (int64_t)sim->n_t_max));
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (n_elems > 0)
        HIP_OR_FAIL(hipMemcpyAsync(dst, sim->traces(), (size_t)n_elems * sizeof(float),
                                   dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(hipStreamSynchronize(st));
    return FW_OK;
}

int fw_reset_state(fw_sim *sim, void *hip_stream)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (!sim->ws) return fail(FW_ESTATE, "no workspace bound");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIP_OR_FAIL(hipMemsetAsync(sim->ws, 0, (size_t)sim->state_end, st));
    HIP_OR_FAIL(hipMemsetAsync(sim->d_step.ptr, 0, sizeof(int64_t), st));
    HIP_OR_FAIL(hipMemsetAsync(static_cast<char *>(sim->d_step.ptr) + sizeof(int64_t), 0xff, sizeof(int64_t), st));
    if (sim->n_rec > 0)
        HIP_OR_FAIL(hipMemsetAsync(sim->traces(), 0, (size_t)sim->n_rec * std::max(sim->n_t_max, 1) * sizeof(float), st));
    sim->host_step = 0;
    return FW_OK;
}

int fw_first_nonfinite_step(fw_sim *sim, int64_t *row, void *hip_stream)
{
    g_err.clear();
    if (!sim || !row) return fail(FW_EINVAL, "NULL argument");
    if (!sim->ws) return fail(FW_ESTATE, "no workspace bound");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIP_OR_FAIL(hipMemcpyAsync(row, static_cast<char *>(sim->d_step.ptr) + sizeof(int64_t), sizeof(int64_t),
                               hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(hipStreamSynchronize(st));
    return FW_OK;
}

int fw_get_step(const fw_sim *sim, int64_t *step)
{
    if (!sim || !step) return fail(FW_EINVAL, "NULL argument");
    *step = sim->host_step;
    return FW_OK;
}

int64_t fw_state_bytes(const fw_sim *sim) { return sim ? sim->state_end + kAlignBytes : -1; }

int fw_save_state(fw_sim *sim, void *d_dst, void *hip_stream)
{
    g_err.clear();
    if (!sim || !d_dst) return fail(FW_EINVAL, "NULL argument");
    if (!sim->ws) return fail(FW_ESTATE, "no workspace bound");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    char *dst = static_cast<char *>(d_dst);
    HIP_OR_FAIL(fw::launch_copy(dst, sim->ws, sim->state_end, st));
    // the step counter and the first non-finite trace row travel together
    HIP_OR_FAIL(hipMemcpyAsync(dst + sim->state_end, sim->d_step.ptr, 2 * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    return FW_OK;
}

int fw_load_state(fw_sim *sim, const void *d_src, void *hip_stream)
{
    g_err.clear();
    if (!sim || !d_src) return fail(FW_EINVAL, "NULL argument");
    if (!sim->ws) return fail(FW_ESTATE, "no workspace bound");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const char *src = static_cast<const char *>(d_src);
    HIP_OR_FAIL(fw::launch_copy(sim->ws, src, sim->state_end, st));
    HIP_OR_FAIL(hipMemcpyAsync(sim->d_step.ptr, src + sim->state_end, 2 * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    int64_t step = 0;
    HIP_OR_FAIL(hipMemcpyAsync(&step, src + sim->state_end, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(hipStreamSynchronize(st));
    sim->host_step = step;
    return FW_OK;
}

int fw_time_kernels(fw_sim *sim, int n_steps, void *hip_stream, double *avg_ms)
{
    g_err.clear();
    if (!sim || !avg_ms) return fail(FW_EINVAL, "NULL argument");
    if (n_steps < 1) return fail(FW_EINVAL, "n_steps must be >= 1");
    if (!sim->ws || !sim->media_set || !sim->table_set) return fail(FW_ESTATE, "set up the simulation first");
    if (sim->tiles_dirty) {
        int rc = build_tiles(sim);
        if (rc != FW_OK) return rc;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const fw::StepArgs a = step_args(sim);
    const fw::SrcRecArgs r = srcrec_args(sim);
    // the launches of one step in the order fw_step issues them, each with
    // the update it belongs to (0 velocity, 1 pressure, 2 sources/receivers)
    std::vector<std::pair<int, fw::StepArgs>> plan;
    if (interleaved_on(sim, a)) {
        for (const auto &L : sim->chunks) {
            const fw::StepArgs c = chunk_args(sim, a, L);
            if (L.vn > 0) plan.emplace_back(0, c);
            if (L.pn > 0) plan.emplace_back(1, c);
        }
    } else {
        plan.emplace_back(0, a);
        plan.emplace_back(1, a);
    }
    plan.emplace_back(2, a);
    const size_t per = plan.size() + 1;
    std::vector<hipEvent_t> ev((size_t)n_steps * per, nullptr);
    for (auto &e : ev) HIP_OR_FAIL(hipEventCreate(&e));
    int rc = FW_OK;
    for (int i = 0; i < n_steps && rc == FW_OK; ++i) {
        hipEvent_t *e = &ev[(size_t)i * per];
        hipError_t err = hipEventRecord(e[0], st);
        for (size_t k = 0; k < plan.size() && err == hipSuccess; ++k) {
            const fw::StepArgs &c = plan[k].second;
            if (plan[k].first == 0)
                err = fw::launch_velocity(sim->ndim, sim->nmech, sim->tile_rows, sim->rows_per_thread, c, st);
            else if (plan[k].first == 1)
                err = fw::launch_pressure(sim->ndim, sim->nmech, sim->tile_rows, sim->rows_per_thread, c, st);
            else
                err = fw::launch_src_rec(r, st);
            if (err == hipSuccess) err = hipEventRecord(e[k + 1], st);
        }
        if (err != hipSuccess) rc = fail(FW_EHIP, "timed launch: %s", hipGetErrorString(err));
    }
    double tot[3] = {0, 0, 0};
    if (rc == FW_OK) {
        hipError_t err = hipStreamSynchronize(st);
        if (err != hipSuccess) rc = fail(FW_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(err));
        for (int i = 0; i < n_steps && rc == FW_OK; ++i)
            for (size_t k = 0; k < plan.size() && rc == FW_OK; ++k) {
                float ms = 0;
                err = hipEventElapsedTime(&ms, ev[(size_t)i * per + k], ev[(size_t)i * per + k + 1]);
                if (err != hipSuccess) rc = fail(FW_EHIP, "hipEventElapsedTime: %s", hipGetErrorString(err));
                tot[plan[k].first] += ms;
            }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (rc != FW_OK) return rc;
    for (int k = 0; k < 3; ++k) avg_ms[k] = tot[k] / n_steps;
    sim->host_step += n_steps;
    return FW_OK;
}


// One step plus the energy diagnostics, with p^n kept in pold (total_cells
// floats) and the per-tile partial sums in partial (n_tiles x 3 doubles).
static int energy_step_impl(fw_sim *sim, double *out, hipStream_t st, float *pold, double *partial)
{
    const fw::StepArgs a = step_args(sim);
    const fw::SrcRecArgs r = srcrec_args(sim);
    HIP_OR_FAIL(fw::launch_velocity(sim->ndim, sim->nmech, sim->tile_rows, sim->rows_per_thread, a, st));
    HIP_OR_FAIL(fw::launch_copy(pold, a.f.p, sim->total_cells * (int64_t)sizeof(float), st));
    HIP_OR_FAIL(fw::launch_pressure(sim->ndim, sim->nmech, sim->tile_rows, sim->rows_per_thread, a, st));
    HIP_OR_FAIL(fw::launch_src_rec(r, st));
    HIP_OR_FAIL(fw::launch_energy(sim->ndim, a, pold, partial, st));
    std::vector<double> part((size_t)sim->n_tiles * 3);
    HIP_OR_FAIL(hipMemcpyAsync(part.data(), partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(hipStreamSynchronize(st));
    for (int d = 0; d < sim->n_domains; ++d) out[3 * d] = out[3 * d + 1] = out[3 * d + 2] = 0.0;
    for (int t = 0; t < sim->n_tiles; ++t) {
        double *o = out + 3 * sim->h_tile_dom[t];
        o[0] += part[3 * (size_t)t];
        o[1] = std::max(o[1], part[3 * (size_t)t + 1]);
        o[2] += part[3 * (size_t)t + 2];
    }
    sim->host_step += 1;
    for (int d = 0; d < sim->n_domains; ++d)
        if (out[3 * d + 2] > 0) return fail(FW_ENONFINITE, "domain %d: %.0f non-finite pressure values", d, out[3 * d + 2]);
    return FW_OK;
}

extern "C" int fw_energy_step(fw_sim *sim, double *out, void *hip_stream)
{
    g_err.clear();
    if (!sim || !out) return fail(FW_EINVAL, "NULL argument");
    if (!sim->ws || !sim->media_set || !sim->table_set) return fail(FW_ESTATE, "set up the simulation first");
    if (sim->tiles_dirty) {
        int rc = build_tiles(sim);
        if (rc != FW_OK) return rc;
    }
    HIP_OR_FAIL(sim->d_pold.ensure((size_t)sim->total_cells * sizeof(float)));
    HIP_OR_FAIL(sim->d_partial.ensure((size_t)sim->n_tiles * 3 * sizeof(double)));
    return energy_step_impl(sim, out, static_cast<hipStream_t>(hip_stream), sim->d_pold.as<float>(),
                            sim->d_partial.as<double>());
}

// Scratch of the allocation-free energy step: p^n of up to kNoAllocCells
// cells, then the partial sums of up to kNoAllocTiles tiles.  Every GPU the
// library runs on holds its own copy until the process ends.
constexpr int64_t kNoAllocCells = int64_t(8) << 20;
constexpr int64_t kNoAllocTiles = int64_t(1) << 16;
constexpr size_t kNoAllocBytes = (size_t)kNoAllocCells * sizeof(float) + (size_t)kNoAllocTiles * 3 * sizeof(double);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices] = {};

// Device address of this GPU's copy of scratch, looked up once per device
// with that device current.  The host-side name of the array is not a device
// address and is never passed to a kernel or a copy.
static int scratch_address(void **ptr)
{
    int dev = -1;
    HIP_OR_FAIL(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FW_EUNSUPPORTED, "device %d is beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(FW_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *ptr = g_scratch_dev[dev];
    return FW_OK;
}

extern "C" int fw_energy_step_noalloc(fw_sim *sim, double *out, void *hip_stream)
{
    g_err.clear();
    if (!sim || !out) return fail(FW_EINVAL, "NULL argument");
    if (!sim->ws || !sim->media_set || !sim->table_set) return fail(FW_ESTATE, "set up the simulation first");
    if (sim->tiles_dirty)
        return fail(FW_ESTATE, "the tile lists are not built yet (building them allocates): take one fw_step or "
                    "fw_energy_step first");
    if (sim->total_cells > kNoAllocCells)
        return fail(FW_EINVAL, "%lld cells (domains padded to 64 cells) exceed the allocation-free limit of %lld",
                    (long long)sim->total_cells, (long long)kNoAllocCells);
    if (sim->n_tiles > kNoAllocTiles)
        return fail(FW_EINVAL, "%d tiles exceed the allocation-free limit of %lld", sim->n_tiles,
                    (long long)kNoAllocTiles);
    void *base = nullptr;
    int rc = scratch_address(&base);
    if (rc != FW_OK) return rc;
    float *pold = static_cast<float *>(base);
    double *partial = reinterpret_cast<double *>(static_cast<char *>(base) + (size_t)kNoAllocCells * sizeof(float));
    return energy_step_impl(sim, out, static_cast<hipStream_t>(hip_stream), pold, partial);
}

// ------------------------------------------------------------------ adjoint --
static int64_t adj_state_stride(const fw_sim *s) { return align_up(s->state_end + 8, kAlignBytes); }

static int adj_layout(const fw_sim *s, int n_steps, int ckpt_every, int64_t *n_ck, int64_t *off_seg, int64_t *off_lam,
                      int64_t *off_scr, int64_t *total)
{
    if (n_steps < 1 || ckpt_every < 1) return fail(FW_EINVAL, "n_steps and ckpt_every must be >= 1");
    const int64_t SB = adj_state_stride(s);
    *n_ck = (n_steps + ckpt_every - 1) / ckpt_every;
    *off_seg = *n_ck * SB;
    *off_lam = *off_seg + (int64_t)(std::min(ckpt_every, n_steps) + 1) * SB;
    *off_scr = *off_lam + SB;
    // scratch: the six pending-derivative fields, then dJ/dK and dJ/ds of
    // fw_adjoint (unpadded layout) before its chain rule
    *total = *off_scr + align_up(2LL * 3 * s->total_cells * 4, kAlignBytes) +
             2 * align_up(s->total_packed * 4, kAlignBytes);
    return FW_OK;
}

extern "C" int64_t fw_adjoint_workspace_bytes(const fw_sim *sim, int n_steps, int ckpt_every)
{
    if (!sim) return -1;
    int64_t nck, os, ol, oc, tot;
    if (adj_layout(sim, n_steps, ckpt_every, &nck, &os, &ol, &oc, &tot) != FW_OK) return -1;
    return tot;
}

static int copy_state(fw_sim *s, char *dst, const char *src, hipStream_t st)
{
    HIP_OR_FAIL(fw::launch_copy(dst, src, s->state_end, st));
    return FW_OK;
}

extern "C" int fw_forward_checkpointed(fw_sim *sim, int n_steps, int ckpt_every, void *d_work, int64_t bytes,
                                       void *hip_stream)
{
    g_err.clear();
    if (!sim || !d_work) return fail(FW_EINVAL, "NULL argument");
    int64_t nck, os, ol, oc, tot;
    int rc = adj_layout(sim, n_steps, ckpt_every, &nck, &os, &ol, &oc, &tot);
    if (rc != FW_OK) return rc;
    if (bytes < tot) return fail(FW_ENOMEM, "adjoint workspace too small: %lld < %lld", (long long)bytes, (long long)tot);
    if ((reinterpret_cast<uintptr_t>(d_work) % kAlignBytes) != 0)
        return fail(FW_EINVAL, "adjoint workspace must be 256-byte aligned");
    if (!sim->ws || !sim->media_set || !sim->table_set) return fail(FW_ESTATE, "set up the simulation first");
    char *w = static_cast<char *>(d_work);
    const int64_t SB = adj_state_stride(sim);
    rc = fw_reset_state(sim, hip_stream);
    if (rc != FW_OK) return rc;
    for (int64_t k = 0; k < nck; ++k) {
        rc = fw_save_state(sim, w + k * SB, hip_stream);
        if (rc != FW_OK) return rc;
        const int n = (int)std::min<int64_t>(ckpt_every, n_steps - k * ckpt_every);
        rc = fw_step(sim, n, hip_stream);
        if (rc != FW_OK) return rc;
    }
    return FW_OK;
}

// The reverse sweep shared by fw_adjoint and fw_adjoint_modulus: accumulates
// dJ/dK into d_grad_K and dJ/ds into d_grad_s (unpadded layout).
static int adjoint_sweep(fw_sim *sim, int n_steps, int ckpt_every, void *d_work, int64_t bytes,
                         const float *d_adj_src, float *d_grad_K, float *d_grad_s, void *hip_stream)
{
    int64_t nck, os, ol, oc, tot;
    int rc = adj_layout(sim, n_steps, ckpt_every, &nck, &os, &ol, &oc, &tot);
    if (rc != FW_OK) return rc;
    if (bytes < tot) return fail(FW_ENOMEM, "adjoint workspace too small: %lld < %lld", (long long)bytes, (long long)tot);
    if ((reinterpret_cast<uintptr_t>(d_work) % kAlignBytes) != 0)
        return fail(FW_EINVAL, "adjoint workspace must be 256-byte aligned");
    if (!sim->ws || !sim->media_set || !sim->table_set) return fail(FW_ESTATE, "set up the simulation first");
    for (double b : sim->beta)
        if (b != 0.0) return fail(FW_EUNSUPPORTED, "the adjoint supports linear media only (beta = 0 in every class)");
    if (sim->amap) return fail(FW_EUNSUPPORTED, "the adjoint does not support a relaxation strength map");
    if (sim->fd_b != 0.0) return fail(FW_EUNSUPPORTED, "the adjoint does not support the widened stencil");
    if (sim->tiles_dirty) {
        rc = build_tiles(sim);
        if (rc != FW_OK) return rc;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    char *w = static_cast<char *>(d_work);
    const int64_t SB = adj_state_stride(sim);
    char *seg = w + os;
    char *lam = w + ol;
    float *scr = reinterpret_cast<float *>(w + oc);
    // the recompute below moves the device step counter; keep its value in
    // the spare bytes after the adjoint state and restore it at the end
    HIP_OR_FAIL(hipMemsetAsync(lam, 0, (size_t)sim->state_end, st));
    HIP_OR_FAIL(hipMemcpyAsync(lam + sim->state_end, sim->d_step.ptr, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    fw::AdjArgs A{};
    A.s = step_args(sim);
    A.lam = fields_at(sim, lam);
    for (int a = 0; a < 3; ++a) {
        A.lamD1[a] = scr + (int64_t)a * sim->total_cells;
        A.lamD2[a] = scr + (int64_t)(3 + a) * sim->total_cells;
    }
    A.gK = d_grad_K;
    A.gs = d_grad_s;
    A.cadj = sim->d_cadj.as<fw::ClassAdj>();
    A.tile_rows = sim->tile_rows;
    A.fold_div = 0;
    fw::AdjInjectArgs J{};
    J.lam_p = A.lam.p;
    J.cells = sim->d_adj_cells.as<int64_t>();
    J.offsets = sim->d_adj_off.as<int32_t>();
    J.rec_index = sim->d_adj_idx.as<int32_t>();
    J.n_cells = sim->n_adj_cells;
    J.res = d_adj_src;
    J.n_rec = sim->n_rec;
    for (int64_t k = nck - 1; k >= 0; --k) {
        const int64_t s0 = k * ckpt_every;
        const int64_t s1 = std::min<int64_t>(s0 + ckpt_every, n_steps);
        // segment states: the checkpoint goes to slot 0 (and the step counter
        // to the device), then each recomputed step reads slot j and writes
        // slot j + 1 directly (no copies)
        rc = copy_state(sim, seg, w + k * SB, st);
        if (rc != FW_OK) return rc;
        HIP_OR_FAIL(hipMemcpyAsync(sim->d_step.ptr, w + k * SB + sim->state_end, sizeof(int64_t),
                                   hipMemcpyDeviceToDevice, st));
        for (int64_t j = 1; j <= s1 - s0; ++j) {
            fw::StepArgs a = step_args(sim);
            a.f = fields_at(sim, seg + (j - 1) * SB);
            a.fo = fields_at(sim, seg + j * SB);
            fw::SrcRecArgs r = srcrec_args(sim);
            r.p = a.fo.p;
            HIP_OR_FAIL(fw::launch_velocity(sim->ndim, sim->nmech, sim->tile_rows, sim->rows_per_thread, a, st));
            HIP_OR_FAIL(fw::launch_pressure(sim->ndim, sim->nmech, sim->tile_rows, sim->rows_per_thread, a, st));
            HIP_OR_FAIL(fw::launch_src_rec(r, st));
        }
        for (int64_t n = s1 - 1; n >= s0; --n) {
            J.step = n;
            if (n < sim->n_t_max) HIP_OR_FAIL(fw::launch_adjoint_inject(J, st));
            A.s.f = fields_at(sim, seg + (n - s0) * SB);
            A.fnext = fields_at(sim, seg + (n - s0 + 1) * SB);
            HIP_OR_FAIL(fw::launch_adjoint_step(sim->ndim, sim->nmech, A, st));
            A.fold_div = 1;
        }
    }
    if (A.fold_div) HIP_OR_FAIL(fw::launch_adjoint_finish(sim->ndim, A, st));
    HIP_OR_FAIL(hipMemcpyAsync(sim->d_step.ptr, lam + sim->state_end, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    return FW_OK;
}

extern "C" int fw_adjoint_modulus(fw_sim *sim, int n_steps, int ckpt_every, void *d_work, int64_t bytes,
                                  const float *d_adj_src, float *d_grad_K, float *d_grad_s, void *hip_stream)
{
    g_err.clear();
    if (!sim || !d_work || !d_adj_src || !d_grad_K || !d_grad_s) return fail(FW_EINVAL, "NULL argument");
    return adjoint_sweep(sim, n_steps, ckpt_every, d_work, bytes, d_adj_src, d_grad_K, d_grad_s, hip_stream);
}

// Time-space coefficients for c_ref (Taylor at 0), with the widened 2D
// stencil's off-axis weight b = r^2 / 24 when `wide`; restores the previous
// set when the stability bound fails.
static int set_stencil(fw_sim *sim, double c_ref, bool wide)
{
    const double r = c_ref * sim->dt / sim->dx;
    double prev[4];
    std::copy(sim->fd, sim->fd + 4, prev);
    const double prev_cref = sim->fd_cref, prev_b = sim->fd_b;
    if (c_ref > 0.0) {
        sim->fd_b = wide ? r * r / 24.0 : 0.0;
        time_space_coefficients(r, sim->fd, 2.0 * (sim->ndim - 1) * sim->fd_b);
    } else {
        std::copy(kFD, kFD + 4, sim->fd);
        sim->fd_b = 0.0;
    }
    sim->fd_cref = c_ref;
    if (sim->media_set) {
        const int rc = stability_check(sim, sim->table_set ? sim->min_kk : 1.0);
        if (rc != FW_OK) {
            std::copy(prev, prev + 4, sim->fd);
            sim->fd_cref = prev_cref;
            sim->fd_b = prev_b;
            return rc;
        }
    }
    sim->drop_graph();            // captured steps hold the previous coefficients
    return FW_OK;
}

extern "C" int fw_set_time_space_stencil(fw_sim *sim, double c_ref)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (!(c_ref >= 0.0) || !std::isfinite(c_ref)) return fail(FW_EINVAL, "c_ref must be finite and >= 0 (got %g)", c_ref);
    const double r = c_ref * sim->dt / sim->dx;
    if (!(r < 1.0)) return fail(FW_EINVAL, "c_ref dt / dx = %g: the time-space coefficients need a Courant number < 1", r);
    return set_stencil(sim, c_ref, false);
}

extern "C" int fw_set_widened_stencil(fw_sim *sim, double c_ref)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (sim->ndim != 2) return fail(FW_EUNSUPPORTED, "the widened stencil is built for 2D grids");
    if (!(c_ref >= 0.0) || !std::isfinite(c_ref)) return fail(FW_EINVAL, "c_ref must be finite and >= 0 (got %g)", c_ref);
    const double r = c_ref * sim->dt / sim->dx;
    if (!(r < 1.0)) return fail(FW_EINVAL, "c_ref dt / dx = %g: the time-space coefficients need a Courant number < 1", r);
    return set_stencil(sim, c_ref, true);
}

extern "C" int fw_get_stencil(const fw_sim *sim, double *coef5)
{
    g_err.clear();
    if (!sim || !coef5) return fail(FW_EINVAL, "NULL argument");
    std::copy(sim->fd, sim->fd + 4, coef5);
    coef5[4] = sim->fd_b;
    return FW_OK;
}

extern "C" int fw_set_class_alpha0(fw_sim *sim, int n_classes, const double *alpha0)
{
    g_err.clear();
    if (!sim || !alpha0) return fail(FW_EINVAL, "NULL argument");
    if (!sim->media_set) return fail(FW_ESTATE, "call fw_set_media first");
    if (n_classes != sim->n_classes) return fail(FW_EINVAL, "n_classes %d != %d of fw_set_media", n_classes, sim->n_classes);
    for (int k = 0; k < n_classes; ++k)
        if (!(alpha0[k] > 0.0) || !std::isfinite(alpha0[k]))
            return fail(FW_EINVAL, "class %d: alpha0 must be finite and > 0 (got %g); a class without attenuation has "
                        "no relaxation strength to scale", k, alpha0[k]);
    sim->alpha0.assign(alpha0, alpha0 + n_classes);
    return FW_OK;
}

extern "C" int fw_adjoint(fw_sim *sim, int n_steps, int ckpt_every, void *d_work, int64_t bytes, const float *d_adj_src,
                          float *d_grad_c, float *d_grad_alpha0, void *hip_stream)
{
    g_err.clear();
    if (!sim || !d_work || !d_adj_src || !d_grad_c) return fail(FW_EINVAL, "NULL argument");
    if (d_grad_alpha0 && (int)sim->alpha0.size() != sim->n_classes)
        return fail(FW_ESTATE, "dJ/dalpha0 needs the class alpha0 values (fw_set_class_alpha0)");
    int64_t nck, os, ol, oc, tot;
    int rc = adj_layout(sim, n_steps, ckpt_every, &nck, &os, &ol, &oc, &tot);
    if (rc != FW_OK) return rc;
    if (bytes < tot) return fail(FW_ENOMEM, "adjoint workspace too small: %lld < %lld", (long long)bytes, (long long)tot);
    if ((reinterpret_cast<uintptr_t>(d_work) % kAlignBytes) != 0)
        return fail(FW_EINVAL, "adjoint workspace must be 256-byte aligned");
    if (!sim->ws || !sim->media_set || !sim->table_set) return fail(FW_ESTATE, "set up the simulation first");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    char *w = static_cast<char *>(d_work);
    const int64_t gbytes = align_up(sim->total_packed * 4, kAlignBytes);
    float *gK = reinterpret_cast<float *>(w + tot - 2 * gbytes);
    float *gs = reinterpret_cast<float *>(w + tot - gbytes);
    HIP_OR_FAIL(hipMemsetAsync(gK, 0, (size_t)(2 * gbytes), st));
    rc = adjoint_sweep(sim, n_steps, ckpt_every, d_work, bytes, d_adj_src, gK, gs, hip_stream);
    if (rc != FW_OK) return rc;
    // per class (2 rho c, 1 / alpha0) in FP64, rounded once
    std::vector<float> chain(2 * (size_t)sim->n_classes);
    for (int k = 0; k < sim->n_classes; ++k) {
        chain[2 * k] = (float)(2.0 * sim->rho[k] * sim->c[k]);
        chain[2 * k + 1] = d_grad_alpha0 ? (float)(1.0 / sim->alpha0[k]) : 0.0f;
    }
    HIP_OR_FAIL(sim->d_chain.ensure(chain.size() * sizeof(float)));
    HIP_OR_FAIL(hipMemcpyAsync(sim->d_chain.ptr, chain.data(), chain.size() * sizeof(float), hipMemcpyHostToDevice, st));
    fw::AdjChainArgs C{};
    C.doms = sim->d_doms.as<fw::DomainDesc>();
    C.n_domains = sim->n_domains;
    C.noise_amp = (float)sim->noise_amp;
    C.cls = fields_of(sim).cls;
    C.chain = sim->d_chain.as<float2>();
    C.gK = gK;
    C.gs = gs;
    C.grad_c = d_grad_c;
    C.grad_a0 = d_grad_alpha0;
    C.n_packed = sim->total_packed;
    HIP_OR_FAIL(fw::launch_adjoint_chain(C, st));
    // the host table must outlive the asynchronous upload
    HIP_OR_FAIL(hipStreamSynchronize(st));
    return FW_OK;
}

int fw_stream_probe(fw_sim *sim, int mode, int order, int reps, void *hip_stream, double *avg_ms)
{
    g_err.clear();
    if (!sim || !avg_ms) return fail(FW_EINVAL, "NULL argument");
    if (!sim->ws || !sim->media_set) return fail(FW_ESTATE, "set up the simulation first");
    if (sim->ndim != 3 || sim->n_domains != 1) return fail(FW_EUNSUPPORTED, "the probe runs on one 3D domain");
    if (mode < 0 || mode > 6 || order < 0 || order > 1 || reps < 1)
        return fail(FW_EINVAL, "mode must be 0..6, order 0..1, reps >= 1");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const fw::Fields f = fields_of(sim);
    const fw::DomainDesc &D = sim->doms[0];
    // modes 3 to 6 read the three per-axis arrays as one interleaved or
    // blocked array: they must lie back to back, each holding at least the
    // stored cells; the 64-cell blocks of modes 5 and 6 must tile them
    const int64_t stored = sim->stored(0);
    if (mode >= 5 && stored % 64 != 0)
        return fail(FW_EUNSUPPORTED, "blocked probe modes need a multiple of 64 stored cells");
    if (mode >= 3 && (sim->off_psi2 - sim->off_psi1[0] < 3 * stored * sim->nmech * (int64_t)sizeof(float) ||
                      sim->off_psi1[0] - sim->off_v[0] < 3 * stored * (int64_t)sizeof(float)))
        return fail(FW_EUNSUPPORTED, "interleaved probe modes need the per-axis arrays back to back");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OR_FAIL(hipEventCreate(&e0));
    HIP_OR_FAIL(hipEventCreate(&e1));
    hipError_t err = fw::launch_stream_probe(sim->nmech, mode, order, f, D.n[0], D.pitch, D.n[1], D.n[2], st);
    if (err == hipSuccess) err = hipEventRecord(e0, st);
    for (int r = 0; r < reps && err == hipSuccess; ++r)
        err = fw::launch_stream_probe(sim->nmech, mode, order, f, D.n[0], D.pitch, D.n[1], D.n[2], st);
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(FW_EHIP, "stream probe: %s", hipGetErrorString(err));
    *avg_ms = ms / reps;
    return FW_OK;
}

int fw_set_strength_map(fw_sim *sim, const float *d_scale, void *hip_stream)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    if (!sim->ws || !sim->media_set) return fail(FW_ESTATE, "call fw_set_media first");
    sim->drop_graph();            // captured steps hold the previous map pointer
    if (!d_scale) {
        sim->amap = nullptr;
        return FW_OK;
    }
    if ((reinterpret_cast<uintptr_t>(d_scale) & 3) != 0) return fail(FW_EINVAL, "the strength map must be 4-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIP_OR_FAIL(sim->d_check.ensure(sizeof(unsigned long long)));
    HIP_OR_FAIL(hipMemsetAsync(sim->d_check.ptr, 0, sizeof(unsigned long long), st));
    HIP_OR_FAIL(fw::launch_count_outside_unit(d_scale, sim->total_packed, sim->d_check.as<unsigned long long>(), st));
    unsigned long long bad = 0;
    HIP_OR_FAIL(hipMemcpyAsync(&bad, sim->d_check.ptr, sizeof(bad), hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(hipStreamSynchronize(st));
    if (bad) {
        sim->amap = nullptr;
        return fail(FW_EINVAL, "%llu strength values are not finite numbers in [0, 1]", bad);
    }
    sim->amap = d_scale;
    return FW_OK;
}

int fw_read_field(fw_sim *sim, int field, int domain, float *dst, int dst_is_device, void *hip_stream)
{
    g_err.clear();
    if (!sim || !dst) return fail(FW_EINVAL, "NULL argument");
    if (!sim->ws) return fail(FW_ESTATE, "no workspace bound");
    if (domain < 0 || domain >= sim->n_domains) return fail(FW_EINVAL, "domain %d out of range", domain);
    const fw::Fields f = fields_of(sim);
    const float *src = nullptr;
    switch (field) {
    case FW_FIELD_P: src = f.p; break;
    case FW_FIELD_VX: src = f.vx; break;
    case FW_FIELD_VY: src = sim->ndim >= 2 ? f.vy : nullptr; break;
    case FW_FIELD_VZ: src = sim->ndim >= 3 ? f.vz : nullptr; break;
    default: break;
    }
    if (!src) return fail(FW_EINVAL, "field %d does not exist in %dD", field, sim->ndim);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const fw::DomainDesc &D = sim->doms[domain];
    HIP_OR_FAIL(hipMemcpy2DAsync(dst, (size_t)D.n[0] * sizeof(float), src + D.cell_off, (size_t)D.pitch * sizeof(float),
                                 (size_t)D.n[0] * sizeof(float), (size_t)(D.n[1] * D.n[2]),
                                 dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(hipStreamSynchronize(st));
    return FW_OK;
}

int fw_device_copy(void *d_dst, const void *d_src, int64_t bytes, void *hip_stream)
{
    g_err.clear();
    if (bytes < 0 || (bytes > 0 && (!d_dst || !d_src))) return fail(FW_EINVAL, "bad copy arguments");
    HIP_OR_FAIL(fw::launch_copy(d_dst, d_src, bytes, static_cast<hipStream_t>(hip_stream)));
    return FW_OK;
}

int fw_set_option(fw_sim *sim, int key, int64_t value)
{
    g_err.clear();
    if (!sim) return fail(FW_EINVAL, "sim is NULL");
    switch (key) {
    case FW_OPT_GRAPH_STEPS:
        if (value < 0 || value > 4096) return fail(FW_EINVAL, "graph steps must be in 0..4096");
        sim->graph_steps = (int)value;
        sim->drop_graph();
        return FW_OK;
    case FW_OPT_MARCH_CHUNK:
        if (value < 0) return fail(FW_EINVAL, "march chunk must be 0 (auto) or >= 1");
        sim->march_chunk = (int)value;
        sim->tiles_dirty = true;
        return FW_OK;
    case FW_OPT_TILE_ROWS:
        if (value != 4 && value != 8 && value != 16) return fail(FW_EINVAL, "tile rows must be 4, 8 or 16");
        if (value == 4 && sim->rows_per_thread == 2) return fail(FW_EINVAL, "4-row tiles use one row per thread");
        sim->tile_rows = (int)value;
        sim->tiles_dirty = true;
        return FW_OK;
    case FW_OPT_PERSISTENT:
        if (value < 0 || value > 64) return fail(FW_EINVAL, "persistent blocks per CU must be in 0..64");
        sim->persistent = (int)value;
        sim->drop_graph();
        return FW_OK;
    case FW_OPT_TILE_ORDER:
        if (value < 0 || value > 2)
            return fail(FW_EINVAL, "tile order must be 0 (x fastest), 1 (y fastest) or 2 (plane-major XCD bands)");
        sim->tile_order = (int)value;
        sim->tiles_dirty = true;
        return FW_OK;
    case FW_OPT_PLANE_KERNELS:
        if (value < -1 || value > 1) return fail(FW_EINVAL, "plane kernels must be -1 (auto), 0 or 1");
        sim->plane_kernels = (int)value;
        sim->tiles_dirty = true;
        return FW_OK;
    case FW_OPT_PLANE_ROWS:
        if (sim->ndim == 2 ? (value != 4 && value != 8 && value != 16) : (value != 4 && value != 8))
            return fail(FW_EINVAL, "plane-kernel tile rows must be 4 or 8 (2D tile kernels: 4, 8 or 16)");
        sim->plane_rows = (int)value;
        sim->tiles_dirty = true;
        return FW_OK;
    case FW_OPT_VEL_PLANES:
        if (value != 1 && value != 2 && value != 4)
            return fail(FW_EINVAL, "velocity plane-kernel tiles hold 1, 2 or 4 planes");
        sim->vel_planes = (int)value;
        sim->tiles_dirty = true;
        return FW_OK;
    case FW_OPT_PRS_PLANES:
        if (value != 2 && value != 4 && value != 8)
            return fail(FW_EINVAL, "pressure plane-kernel tiles hold 2, 4 or 8 planes");
        sim->prs_planes = (int)value;
        sim->tiles_dirty = true;
        return FW_OK;
    case FW_OPT_STEP_CHUNK:
        if (value != -1 && value != 0 && (value < 4 || value > 65536))
            return fail(FW_EINVAL, "interleaved chunk must be -1 (auto), 0 (off) or 4..65536 planes");
        sim->step_chunk = (int)value;
        sim->tiles_dirty = true;
        return FW_OK;
    case FW_OPT_RESIDENT_1D:
        if (value < -1 || value > 1) return fail(FW_EINVAL, "resident 1D step must be -1 (auto), 0 (off) or 1");
        sim->resident = (int)value;
        sim->drop_graph();
        return FW_OK;
    case FW_OPT_ROWS_PER_THREAD:
        if (value != 1 && value != 2) return fail(FW_EINVAL, "rows per thread must be 1 or 2");
        if (value == 2 && sim->tile_rows == 4) return fail(FW_EINVAL, "4-row tiles use one row per thread");
        sim->rows_per_thread = (int)value;
        sim->drop_graph();
        return FW_OK;
    default:
        return fail(FW_EINVAL, "unknown option %d", key);
    }
}

}  // extern "C"
