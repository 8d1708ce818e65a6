// Host side of the C ABI declared in include/msf.h: argument validation,
// plan/workspace management, layout conversion at the boundary, and the
// batched CG driver of the proximal map (paper Sec. III, eq. (4)).
#include "msf_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <new>

int64_t vol_chunk();
hipError_t cnn_io_buffers(msf_cnn *C, int64_t n, float **g, float **x);

namespace {
thread_local std::string g_err;

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

template <class T>
hipError_t dalloc(T **p, size_t count, int64_t &total)
{
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    total += (int64_t)bytes;
    return hipMalloc((void **)p, bytes);
}

void free_plan_memory(msf_plan *P)
{
    if (P->graph) (void)hipGraphExecDestroy(P->graph);
    P->graph = nullptr;
    P->graph_valid = false;
    void *ptrs[] = {P->d_cs, P->d_rzp, P->d_imtab, P->d_cell_hdr, P->d_cell_ent, P->d_walk_head, P->d_walk_ent, P->d_scale, P->part_g, P->d_cols, P->d_view_offset, P->d_tile_offset, P->x, P->r, P->p, P->bp, P->z64, P->x64, P->vin,
                    P->sy, P->slam, P->sz, P->part_proj, P->part_vol, P->scal, P->iscal, P->consts,
                    P->flags};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (P->host_stage) (void)hipHostFree(P->host_stage);
    P->host_stage = nullptr;
    for (hipEvent_t e : P->ev)
        if (e) (void)hipEventDestroy(e);
    P->ev.clear();
}

// Detector rows that can meet the volume: a ray of row v has height
// z = v_pos * t / L_xy at xy distance t from the source; inside the volume's
// bounding cylinder t >= src_iso - r_max, so rows beyond the bound below stay
// outside the z slab along their whole length (their matrix rows are empty).
void row_range(msf_plan &P)
{
    const double rmax = std::sqrt(0.25 * P.nx * P.nx + 0.25 * P.ny * P.ny);
    const double umax = 0.5 * (P.nu - 1) * P.du + std::fabs(P.offu);
    const double lmax = std::sqrt(P.rsd * P.rsd + umax * umax);
    const double bound = 0.5 * P.nz * lmax / (P.rs - rmax) + 1e-6 * P.nz + P.dv;
    P.iv_lo = 0;
    P.iv_hi = -1;
    int lo = -1, hi = -1;
    for (int iv = 0; iv < P.nv; ++iv) {
        const double zp = (iv - 0.5 * (P.nv - 1)) * P.dv + P.offv;
        if (std::fabs(zp) <= bound) {
            if (lo < 0) lo = iv;
            hi = iv;
        }
    }
    if (lo >= 0) {
        P.iv_lo = lo;
        P.iv_hi = hi;
    }
    // |dz/ds| = |v| / L_xy <= |v| / src_det; a piece inside one xy cell is at most
    // sqrt(2) long in s, so below this slope it crosses at most one z plane
    const double vmax = std::max(std::fabs((P.iv_lo - 0.5 * (P.nv - 1)) * P.dv + P.offv),
                                 std::fabs((P.iv_hi - 0.5 * (P.nv - 1)) * P.dv + P.offv));
    P.steep = vmax / P.rsd * std::sqrt(2.0) >= 0.999;
    // Detector rows whose ray meets one voxel (height 1) inside one xy piece:
    // the ray's detector height per unit z is k = l_xy / d (d = xy distance from
    // the source >= src_iso - r_max), so over the voxel and the piece (at most
    // sqrt(2) long) zp spans at most k_max + (nz / 2) |k_b - k_a| with k_max =
    // lmax / dmin and |k_b - k_a| <= lmax sqrt(2) / dmin^2.  Below two rows
    // (with the gather's 2e-3 widening) every voxel meets at most two
    // consecutive rows per piece, the two candidates the gather always reads.
    const double dmin = P.rs - rmax;
    const double span = (lmax / dmin + 0.5 * P.nz * lmax * std::sqrt(2.0) / (dmin * dmin)) / P.dv + 2e-3;
    P.multi_row = span >= 1.9;
}

// Rays per lane: one wave covers all rows of a detector column that can meet
// the volume, in as few 64-row passes as possible.
int default_rays_per_lane(const msf_plan &P)
{
    if (P.steep) return 1;   // the general z walk runs one ray per lane
    const int rows = P.iv_hi - P.iv_lo + 1;
    const int need = (rows + 63) / 64;
    return std::min(std::max(need, 1), 6);
}

// Per (view, xy cell) piece table of the table-driven voxel adjoint, built once
// (memory: n_views * nx * ny * (4 + 32 K) bytes, K = 2 or 3).  K bounds the detector
// columns that can meet one cell: the cell's width (at most sqrt 2) magnified
// from its nearest possible depth, in columns, plus the 1e-3 slack of the range.
msf_status ensure_cell_table(msf_plan &P)
{
    if (P.d_cell_hdr) return MSF_OK;
    const double rmax = std::sqrt(0.25 * P.nx * P.nx + 0.25 * P.ny * P.ny);
    const double span = std::sqrt(2.0) * P.rsd / ((P.rs - rmax) * P.du) + 2e-3;
    const int k_geom = (int)std::floor(span) + 1;
    if (k_geom > 3) {
        set_error("cell table: more than 3 detector columns can meet a cell on this geometry");
        return MSF_EINVAL;
    }
    P.cell_k = std::max(k_geom, 2);
    const int64_t n = P.n_views * (int64_t)P.nx * P.ny;
    hipError_t e;
    if ((e = dalloc(&P.d_cell_hdr, (size_t)std::max<int64_t>(n, 1), P.workspace_bytes)) != hipSuccess)
        return hip_fail(e, "hipMalloc cell table");
    if ((e = dalloc(&P.d_cell_ent, (size_t)std::max<int64_t>(n * P.cell_k, 1), P.workspace_bytes)) != hipSuccess) {
        (void)hipFree(P.d_cell_hdr);
        P.d_cell_hdr = nullptr;
        return hip_fail(e, "hipMalloc cell table");
    }
    // the forward projector's column walks: (n_views * nu) * (8 + 8 (nx + ny + 2)) bytes
    const int64_t ncol = P.n_views * (int64_t)P.nu;
    if ((e = dalloc(&P.d_walk_head, (size_t)std::max<int64_t>(ncol, 1), P.workspace_bytes)) != hipSuccess ||
        (e = dalloc(&P.d_walk_ent, (size_t)std::max<int64_t>(ncol * (P.nx + P.ny + 2), 1), P.workspace_bytes)) != hipSuccess) {
        for (void *q : {(void *)P.d_cell_hdr, (void *)P.d_cell_ent, (void *)P.d_walk_head, (void *)P.d_walk_ent})
            if (q) (void)hipFree(q);
        P.d_cell_hdr = nullptr;
        P.d_cell_ent = nullptr;
        P.d_walk_head = nullptr;
        P.d_walk_ent = nullptr;
        return hip_fail(e, "hipMalloc walk table");
    }
    if ((e = launch_walk_table(P, nullptr)) != hipSuccess) return hip_fail(e, "walk table");
    int32_t overflow = 0;
    if ((e = hipMemset(P.flags + 4, 0, sizeof(int32_t))) != hipSuccess || (e = launch_cell_table(P, nullptr)) != hipSuccess ||
        (e = hipMemcpy(&overflow, P.flags + 4, sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "cell table");
    if (overflow) {
        set_error("cell table: more detector columns meet a cell than the geometry bound allows");
        return MSF_EINVAL;
    }
    return MSF_OK;
}

msf_status setup_tiles(msf_plan &P)
{
    // where a ray can cross two z planes inside one xy cell the projector runs the
    // general z walk, compiled for one ray per lane only: the tiles follow it
    if (P.steep) P.tiles.rays_per_lane = 1;
    if (P.tiles.back_mode == 2) {
        const msf_status st = ensure_cell_table(P);
        if (st != MSF_OK) return st;
    }
    const int rpc = 64 * P.tiles.rays_per_lane;
    const int64_t n_ug = (P.nu + P.tiles.waves_per_group - 1) / P.tiles.waves_per_group;
    const int64_t n_vc = P.iv_hi >= P.iv_lo ? (P.iv_hi - P.iv_lo + rpc) / rpc : 0;
    P.tile_offset.assign(P.nf + 1, 0);
    for (int f = 0; f <= P.nf; ++f) P.tile_offset[f] = P.view_offset[f] * n_ug * n_vc;
    const int64_t total = P.tile_offset.back();
    if (total > 0x7fffffffLL) {
        set_error("projector tile count exceeds the grid limit");
        return MSF_EINVAL;
    }
    hipError_t e;
    if (P.d_tile_offset) (void)hipFree(P.d_tile_offset);
    if (P.part_proj) (void)hipFree(P.part_proj);
    if (P.part_g) (void)hipFree(P.part_g);
    P.d_tile_offset = nullptr;
    P.part_proj = nullptr;
    P.part_g = nullptr;
    int64_t dummy = 0;
    if ((e = dalloc(&P.d_tile_offset, P.nf + 1, dummy)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = dalloc(&P.part_proj, (size_t)total, dummy)) != hipSuccess) return hip_fail(e, "hipMalloc");
    // workgroup partials of the fused gather + CG update (same tiling as launch_back_gather)
    P.part_g_per_frame = P.proj_params(false).g_tiles_per_frame;
    if ((e = dalloc(&P.part_g, (size_t)(P.part_g_per_frame * P.nf), dummy)) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipMemcpy(P.d_tile_offset, P.tile_offset.data(), sizeof(int64_t) * (P.nf + 1),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy");
    if (P.graph) (void)hipGraphExecDestroy(P.graph);
    P.graph = nullptr;
    P.graph_valid = false;
    return MSF_OK;
}

bool tiles_ok(const msf_tiles &t)
{
    return (t.rays_per_lane >= 1 && t.rays_per_lane <= 6) &&
           (t.waves_per_group == 1 || t.waves_per_group == 2 || t.waves_per_group == 4) &&
           (t.back_mode >= 0 && t.back_mode <= 2) && (t.xcd_remap == 0 || t.xcd_remap == 1);
}

#define HIPCHK(expr)                                         \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

}  // namespace

// internal volume [f][ny][nx][nz] <-> public [f][nz][ny][nx]
hipError_t vol_to_internal(const msf_plan &P, const float *in, float *out, int check, int32_t *flag, hipStream_t s)
{
    return launch_transpose(in, out, P.nf, P.nz, P.ny * P.nx, check, flag, s);
}
hipError_t vol_to_public(const msf_plan &P, const float *in, float *out, hipStream_t s)
{
    return launch_transpose(in, out, P.nf, P.ny * P.nx, P.nz, 0, nullptr, s);
}
// internal sinogram [view][nu][nv] <-> public [view][nv][nu]
hipError_t sino_to_internal(const msf_plan &P, const float *in, float *out, int check, int32_t *flag, hipStream_t s)
{
    return launch_transpose(in, out, P.n_views, P.nv, P.nu, check, flag, s);
}
hipError_t sino_to_public(const msf_plan &P, const float *in, float *out, hipStream_t s)
{
    return launch_transpose(in, out, P.n_views, P.nu, P.nv, 0, nullptr, s);
}

void set_error(const std::string &msg) { g_err = msg; }

msf_status hip_fail(hipError_t e, const char *where)
{
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? MSF_ENOMEM : MSF_EHIP;
}

extern "C" {

const char *msf_last_error(void) { return g_err.c_str(); }

const char *msf_version(void) { return "msf 0.1 (gfx950)"; }

void msf_solve_opts_default(msf_solve_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-6;
    o->max_iter = 1000;
    o->check_every = 8;
    o->x0_mode = MSF_X0_V;
    o->use_graph = 1;
    o->true_residual = 0;
}

msf_status msf_plan_create(const msf_geometry *g, msf_plan **out)
{
    g_err.clear();
    if (!g || !out) { set_error("null geometry or output pointer"); return MSF_EINVAL; }
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->n_frames <= 0 || g->nu <= 0 || g->nv <= 0) {
        set_error("sizes must be positive"); return MSF_EINVAL;
    }
    if ((int64_t)g->nx * g->ny * g->nz > 0x7fffffffLL || (int64_t)g->nu * g->nv > 0x7fffffffLL) {
        set_error("per-frame volume or per-view detector exceeds 2^31 elements"); return MSF_EINVAL;
    }
    if (!finite_pos(g->du) || !finite_pos(g->dv) || !finite_pos(g->src_iso) || !finite_pos(g->src_det) ||
        !std::isfinite(g->det_off_u) || !std::isfinite(g->det_off_v)) {
        set_error("pitches and distances must be positive and finite"); return MSF_EINVAL;
    }
    const double rmax = std::sqrt(0.25 * g->nx * g->nx + 0.25 * g->ny * g->ny);
    if (!(g->src_iso > rmax) || !(g->src_det > g->src_iso + rmax)) {
        set_error("source and detector must lie outside the volume's bounding cylinder"); return MSF_EINVAL;
    }
    if (!g->view_offset || g->view_offset[0] != 0) { set_error("view_offset must start at 0"); return MSF_EINVAL; }
    for (int f = 0; f < g->n_frames; ++f)
        if (g->view_offset[f + 1] < g->view_offset[f]) { set_error("view_offset must be non-decreasing"); return MSF_EINVAL; }
    const int64_t nviews = g->view_offset[g->n_frames];
    if (nviews > 0 && !g->angles) { set_error("null angles"); return MSF_EINVAL; }
    for (int64_t i = 0; i < nviews; ++i)
        if (!std::isfinite(g->angles[i])) { set_error("non-finite angle"); return MSF_EINVAL; }

    msf_plan *P = new (std::nothrow) msf_plan();
    if (!P) { set_error("host allocation failed"); return MSF_ENOMEM; }
    P->nx = g->nx; P->ny = g->ny; P->nz = g->nz; P->nf = g->n_frames; P->nu = g->nu; P->nv = g->nv;
    P->du = g->du; P->dv = g->dv; P->rs = g->src_iso; P->rsd = g->src_det;
    P->offu = g->det_off_u; P->offv = g->det_off_v;
    P->view_offset.assign(g->view_offset, g->view_offset + g->n_frames + 1);
    P->angles.assign(g->angles, g->angles + nviews);
    P->n_views = nviews;
    P->nvox = (int64_t)g->nx * g->ny * g->nz;
    P->nvox_total = P->nvox * g->n_frames;
    P->nmeas_total = nviews * (int64_t)g->nu * g->nv;
    P->vol_blocks_per_frame = (P->nvox + vol_chunk() - 1) / vol_chunk();
    row_range(*P);
    P->tiles.rays_per_lane = default_rays_per_lane(*P);
    P->tiles.waves_per_group = 4;
    P->tiles.back_mode = 2;
    P->tiles.xcd_remap = 1;

    auto fail = [&](msf_status st) { free_plan_memory(P); delete P; return st; };
    hipError_t e;
    int64_t &tot = P->workspace_bytes;
    std::vector<double2> cs(std::max<int64_t>(nviews, 1));
    for (int64_t i = 0; i < nviews; ++i) cs[i] = make_double2(std::cos(P->angles[i]), std::sin(P->angles[i]));
    if ((e = dalloc(&P->d_cs, (size_t)std::max<int64_t>(nviews, 1), tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = dalloc(&P->d_view_offset, P->nf + 1, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = dalloc(&P->d_rzp, (size_t)P->nv, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = dalloc(&P->d_cols, (size_t)std::max<int64_t>(nviews * P->nu, 1), tot)) != hipSuccess)
        return fail(hip_fail(e, "hipMalloc"));
    std::vector<double2> rzp(P->nv);
    for (int iv = 0; iv < P->nv; ++iv) {
        const double zp = (iv - 0.5 * (P->nv - 1)) * P->dv + P->offv;
        // a huge finite 1/zp for the level ray lets the adjoint use one crossing formula for every row
        rzp[iv] = make_double2(zp, zp != 0.0 ? 1.0 / zp : 1e290);
    }
    // 3D length per unit of xy length of the ray of pixel (u, v): sqrt(1 + (zp / lxy)^2), lxy = |pixel - source|_xy
    // z-plane crossing slope of the ray of pixel (u, v): s = (k - nz/2) lxy / zp - sf, used by every kernel
    if ((e = dalloc(&P->d_scale, (size_t)P->nu * P->nv, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = dalloc(&P->d_imtab, (size_t)P->nu * P->nv, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    {
        std::vector<float> sc((size_t)P->nu * P->nv);
        std::vector<double> im((size_t)P->nu * P->nv);
        for (int iu = 0; iu < P->nu; ++iu) {
            const double u = (iu - 0.5 * (P->nu - 1)) * P->du + P->offu;
            const double lxy = std::sqrt(P->rsd * P->rsd + u * u);
            for (int iv = 0; iv < P->nv; ++iv) {
                const double m = rzp[iv].x / lxy;
                sc[(size_t)iu * P->nv + iv] = (float)std::sqrt(1.0 + m * m);
                im[(size_t)iu * P->nv + iv] = lxy * rzp[iv].y;
            }
        }
        if ((e = hipMemcpy(P->d_scale, sc.data(), sizeof(float) * sc.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return fail(hip_fail(e, "hipMemcpy"));
        if ((e = hipMemcpy(P->d_imtab, im.data(), sizeof(double) * im.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return fail(hip_fail(e, "hipMemcpy"));
    }
    if ((e = hipMemcpy(P->d_rzp, rzp.data(), sizeof(double2) * P->nv, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_fail(e, "hipMemcpy"));
    float **vols[] = {&P->x, &P->r, &P->p, &P->vin};
    for (float **v : vols)
        if ((e = dalloc(v, (size_t)P->nvox_total, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc volume"));
    if ((e = dalloc(&P->bp, (size_t)P->nvox_total, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc volume"));
    float **sinos[] = {&P->sy, &P->slam, &P->sz};
    for (float **v : sinos)
        if ((e = dalloc(v, (size_t)P->nmeas_total, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc sinogram"));
    if ((e = dalloc(&P->part_vol, (size_t)(P->nf * P->vol_blocks_per_frame), tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = dalloc(&P->scal, (size_t)SC_COUNT * P->nf, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = dalloc(&P->iscal, (size_t)IS_COUNT * P->nf, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = dalloc(&P->consts, 4, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = dalloc(&P->flags, 8, tot)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    P->host_stage_bytes = sizeof(double) * (SC_COUNT * P->nf + 8) + sizeof(int32_t) * (IS_COUNT * P->nf + 8);
    if ((e = hipHostMalloc(&P->host_stage, P->host_stage_bytes, hipHostMallocDefault)) != hipSuccess)
        return fail(hip_fail(e, "hipHostMalloc"));
    if ((e = hipMemcpy(P->d_cs, cs.data(), sizeof(double2) * cs.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_fail(e, "hipMemcpy"));
    if ((e = hipMemcpy(P->d_view_offset, P->view_offset.data(), sizeof(int64_t) * (P->nf + 1), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_fail(e, "hipMemcpy"));
    // sinogram rows outside [iv_lo, iv_hi] are never written by the kernels: keep them zero
    for (float **v : sinos)
        if ((e = hipMemset(*v, 0, sizeof(float) * std::max<int64_t>(P->nmeas_total, 1))) != hipSuccess)
            return fail(hip_fail(e, "hipMemset"));
    if ((e = hipMemset(P->bp, 0, sizeof(double) * std::max<int64_t>(P->nvox_total, 1))) != hipSuccess)
        return fail(hip_fail(e, "hipMemset"));
    if ((e = launch_col_table(*P, nullptr)) != hipSuccess) return fail(hip_fail(e, "column table"));
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(hip_fail(e, "hipDeviceSynchronize"));
    msf_status st = setup_tiles(*P);   // after the column table: the cell table is built from it
    if (st != MSF_OK && P->tiles.back_mode == 2) {
        // no room for the cell table: the on-the-fly voxel-driven adjoint needs none
        P->tiles.back_mode = 1;
        set_error("");
        st = setup_tiles(*P);
    }
    if (st != MSF_OK) return fail(st);
    *out = P;
    return MSF_OK;
}

void msf_plan_destroy(msf_plan *P)
{
    if (!P) return;
    (void)hipDeviceSynchronize();
    free_plan_memory(P);
    delete P;
}

msf_status msf_plan_set_tiles(msf_plan *P, const msf_tiles *t)
{
    g_err.clear();
    if (!P || !t) { set_error("null argument"); return MSF_EINVAL; }
    if (!tiles_ok(*t)) { set_error("unsupported tile shape"); return MSF_EINVAL; }
    const msf_tiles old = P->tiles;
    P->tiles = *t;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    msf_status st = setup_tiles(*P);
    if (st != MSF_OK) {
        P->tiles = old;
        setup_tiles(*P);
    }
    return st;
}

msf_status msf_plan_autotune(msf_plan *P, const char *cache_path, msf_tiles *chosen, void *stream)
{
    g_err.clear();
    if (!P) { set_error("null plan"); return MSF_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    hipDeviceProp_t prop;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    // geometry key: sizes, distances and a hash of the angle list
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *d, size_t n) {
        const unsigned char *c = (const unsigned char *)d;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    mix(P->view_offset.data(), P->view_offset.size() * sizeof(int64_t));
    mix(P->angles.data(), P->angles.size() * sizeof(double));
    char key[512];
    snprintf(key, sizeof(key), "%s %d %d %d %d %d %d %.6g %.6g %.6g %.6g %.6g %.6g %016llx", prop.gcnArchName, P->nx,
             P->ny, P->nz, P->nf, P->nu, P->nv, P->du, P->dv, P->rs, P->rsd, P->offu, P->offv, (unsigned long long)h);
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char line[768];
            while (fgets(line, sizeof(line), f)) {
                const size_t kl = strlen(key);
                msf_tiles t{};
                if (strncmp(line, key, kl) == 0 &&
                    sscanf(line + kl, " %d %d %d %d", &t.rays_per_lane, &t.waves_per_group, &t.back_mode,
                           &t.xcd_remap) == 4 && tiles_ok(t)) {
                    fclose(f);
                    msf_status st = msf_plan_set_tiles(P, &t);
                    if (st == MSF_OK && chosen) *chosen = P->tiles;   // as the plan keeps it
                    return st;
                }
            }
            fclose(f);
        }
    }
    // time every shape on a fixed pseudo-random volume (internal buffers)
    HIPCHK(launch_fill(P->p, P->nvox_total, 0.01f, s));
    HIPCHK(launch_fill(P->slam, P->nmeas_total, 1.0f, s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto time_it = [&](auto &&fn, int reps = 3) -> float {
        float best = 1e30f;
        for (int rep = 0; rep < reps; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess || fn() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess)
                return 1e30f;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) best = std::min(best, ms);   // the first run warms caches and code; best of the rest
        }
        return best;
    };
    const msf_tiles old = P->tiles;
    msf_tiles best = old;
    float best_t = 1e30f;
    std::vector<std::pair<float, msf_tiles>> cand;   // every timed (forward + voxel-driven adjoint) shape
    const int R[] = {1, 2, 3, 4, 5, 6}, W[] = {1, 2, 4};
    const int need = (P->iv_hi - P->iv_lo + 64) / 64;
    // forward + voxel-driven adjoint over every shape
    for (int xr = 0; xr <= 1; ++xr)
        for (int w : W)
            for (int r : R) {
                if (r > std::max(need, 1) + 1) continue;   // more rays per lane than rows: idle lanes
                if (P->steep && r != 1) continue;          // steep plans run one ray per lane
                msf_tiles t{r, w, 1, xr};
                P->tiles = t;
                if (setup_tiles(*P) != MSF_OK) continue;
                const float tf = time_it([&] { return launch_forward(*P, PM_WEIGHTED, P->p, nullptr, P->sz, false, s); });
                const float tg = time_it([&] { return launch_back(*P, P->sz, P->bp, false, s); });
                cand.push_back({tf + tg, t});
                P->tiles.back_mode = 2;
                if (setup_tiles(*P) != MSF_OK) continue;
                // back_mode 2 also switches the forward to its walk table: time both again
                const float tf2 = time_it([&] { return launch_forward(*P, PM_WEIGHTED, P->p, nullptr, P->sz, false, s); });
                const float tt = time_it([&] { return launch_back(*P, P->sz, P->bp, false, s); });
                t.back_mode = 2;
                cand.push_back({tf2 + tt, t});
            }
    // the closest shapes often differ by less than the spread of two runs: time the
    // three fastest again, the best of five runs each, and keep the fastest of those
    std::sort(cand.begin(), cand.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    for (size_t i = 0; i < std::min<size_t>(cand.size(), 3); ++i) {
        P->tiles = cand[i].second;
        if (cand[i].first >= 1e30f || setup_tiles(*P) != MSF_OK) continue;
        const float tf = time_it([&] { return launch_forward(*P, PM_WEIGHTED, P->p, nullptr, P->sz, false, s); }, 6);
        const float tb = time_it([&] { return launch_back(*P, P->sz, P->bp, false, s); }, 6);
        if (tf + tb < best_t) { best_t = tf + tb; best = cand[i].second; }
    }
    // the ray-driven scatter adjoint at the best shape (it shares the forward's tiling)
    if (best_t < 1e30f) {
        P->tiles = best;
        P->tiles.back_mode = 0;
        if (setup_tiles(*P) == MSF_OK) {
            const float tf = time_it([&] { return launch_forward(*P, PM_WEIGHTED, P->p, nullptr, P->sz, false, s); });
            const float ts = time_it([&] {
                hipError_t e = launch_fill_d(P->bp, P->nvox_total, s);
                return e != hipSuccess ? e : launch_back(*P, P->sz, P->bp, false, s);
            });
            if (tf + ts < best_t) { best_t = tf + ts; best.back_mode = 0; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(launch_fill_d(P->bp, P->nvox_total, s));   // the solver expects a cleared accumulator
    P->tiles = best;
    msf_status st = setup_tiles(*P);
    if (st != MSF_OK) return st;
    HIPCHK(hipStreamSynchronize(s));
    if (chosen) *chosen = P->tiles;
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "a")) {
            fprintf(f, "%s %d %d %d %d\n", key, best.rays_per_lane, best.waves_per_group, best.back_mode, best.xcd_remap);
            fclose(f);
        }
    }
    (void)old;
    return MSF_OK;
}

msf_status msf_plan_get_tiles(const msf_plan *P, msf_tiles *t)
{
    if (!P || !t) { set_error("null argument"); return MSF_EINVAL; }
    *t = P->tiles;
    return MSF_OK;
}

msf_status msf_plan_sizes(const msf_plan *P, int64_t *nv, int64_t *nm, int64_t *wb)
{
    if (!P) { set_error("null plan"); return MSF_EINVAL; }
    if (nv) *nv = P->nvox_total;
    if (nm) *nm = P->nmeas_total;
    if (wb) *wb = P->workspace_bytes;
    return MSF_OK;
}

msf_status msf_project(msf_plan *P, const float *x, float *y, void *stream)
{
    g_err.clear();
    if (!P || !x || !y) { set_error("null argument"); return MSF_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(vol_to_internal(*P, x, P->p, 0, nullptr, s));
    // rows that cannot meet the volume are not traced: they must read as zero
    HIPCHK(launch_fill(P->sz, P->nmeas_total, 0.0f, s));
    HIPCHK(launch_forward(*P, PM_PLAIN, P->p, nullptr, P->sz, false, s));
    HIPCHK(sino_to_public(*P, P->sz, y, s));
    return MSF_OK;
}

msf_status msf_backproject(msf_plan *P, const float *y, float *x, void *stream)
{
    g_err.clear();
    if (!P || !x || !y) { set_error("null argument"); return MSF_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(sino_to_internal(*P, y, P->sz, 0, nullptr, s));
    HIPCHK(launch_prescale(*P, P->sz, s));
    HIPCHK(launch_fill_d(P->bp, P->nvox_total, s));
    HIPCHK(launch_back(*P, P->sz, P->bp, false, s));
    HIPCHK(launch_d2f(P->bp, P->p, P->nvox_total, s));
    HIPCHK(vol_to_public(*P, P->p, x, s));
    HIPCHK(launch_fill_d(P->bp, P->nvox_total, s));
    return MSF_OK;
}

msf_status msf_plan_set_timing(msf_plan *P, int32_t enable)
{
    g_err.clear();
    if (!P) { set_error("null plan"); return MSF_EINVAL; }
    HIPCHK(hipDeviceSynchronize());
    P->timing = enable != 0;
    P->t_fwd_ms = P->t_back_ms = 0.0;
    P->n_fwd = P->n_back = 0;
    return MSF_OK;
}

msf_status msf_plan_get_timing(const msf_plan *P, msf_timing *t)
{
    if (!P || !t) { set_error("null argument"); return MSF_EINVAL; }
    t->forward_ms = P->t_fwd_ms;
    t->forward_launches = P->n_fwd;
    t->back_ms = P->t_back_ms;
    t->back_launches = P->n_back;
    return MSF_OK;
}

msf_status msf_count_intersections(msf_plan *P, int64_t *per_frame, void *stream)
{
    g_err.clear();
    if (!P || !per_frame) { set_error("null argument"); return MSF_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(launch_forward(*P, PM_COUNT, P->p, nullptr, P->sz, false, s));
    std::vector<float> h((size_t)std::max<int64_t>(P->nmeas_total, 1));
    HIPCHK(hipMemcpyAsync(h.data(), P->sz, sizeof(float) * P->nmeas_total, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t per_view = (int64_t)P->nu * P->nv;
    for (int f = 0; f < P->nf; ++f) {
        int64_t c = 0;
        for (int64_t i = P->view_offset[f] * per_view; i < P->view_offset[f + 1] * per_view; ++i) c += (int64_t)h[i];
        per_frame[f] = c;
    }
    return MSF_OK;
}

namespace {

// Transposes and checks the inputs, then computes ||b|| and r = b - H x for the
// chosen start (v or a caller's x0).  Validation finishes before anything is
// written to caller memory.
// tol: the recursive residual at which CG steps freeze a frame; tol_final:
// the FP64 residual at which a refined solve accepts it (refinement only).
msf_status prepare(msf_plan *P, const float *v, const float *y, const float *lam, double sigma, double tol,
                   int max_iter, const float *x0_user, hipStream_t s, double tol_final = 0.0)
{
    double *hc = (double *)P->host_stage;
    int32_t *hflags = (int32_t *)(hc + 4);
    hc[0] = 1.0 / (sigma * sigma);
    hc[1] = tol;
    hc[2] = (double)max_iter;
    hc[3] = tol_final;
    HIPCHK(hipMemcpyAsync(P->consts, hc, 4 * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(P->flags, 0, 4 * sizeof(int32_t), s));
    HIPCHK(vol_to_internal(*P, v, P->vin, 1, P->flags + 2, s));
    HIPCHK(sino_to_internal(*P, y, P->sy, 1, P->flags + 1, s));
    HIPCHK(sino_to_internal(*P, lam, P->slam, 2, P->flags + 0, s));
    if (x0_user) HIPCHK(vol_to_internal(*P, x0_user, P->x, 1, P->flags + 3, s));
    else HIPCHK(launch_copy(P->x, P->vin, P->nvox_total, s));
    HIPCHK(hipMemcpyAsync(hflags, P->flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hflags[0] || hflags[1] || hflags[2] || hflags[3]) {
        set_error("invalid input: " + std::to_string(hflags[0]) + " negative/non-finite lambda, " +
                  std::to_string(hflags[1]) + " non-finite y, " + std::to_string(hflags[2]) + " non-finite v, " +
                  std::to_string(hflags[3]) + " non-finite x0");
        return MSF_EINVAL;
    }
    // ||b|| with b = A^T Lambda y + v / sigma^2
    HIPCHK(launch_sino_mul_scaled(P->slam, P->sy, P->d_scale, (int64_t)P->nu * P->nv, P->sz, P->nmeas_total, s));
    HIPCHK(launch_back(*P, P->sz, P->bp, false, s));
    HIPCHK(launch_vol_bnorm(*P, s));
    HIPCHK(launch_scalar_reduce(*P, RW_BNORM, s));
    // r = b - H x0, p = r
    HIPCHK(launch_forward(*P, PM_RESID, P->x, P->sy, P->sz, false, s));
    HIPCHK(launch_back(*P, P->sz, P->bp, false, s));
    HIPCHK(launch_vol_init_residual(*P, s));
    HIPCHK(launch_scalar_reduce(*P, RW_INIT, s));
    return MSF_OK;
}

// host copy of the per-frame relative residual of the start (SC_REL right after setup)
msf_status start_residual(msf_plan *P, std::vector<double> &out, hipStream_t s)
{
    out.assign(P->nf, 0.0);
    HIPCHK(hipMemcpyAsync(out.data(), P->scal + SC_REL * P->nf, sizeof(double) * P->nf, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MSF_OK;
}

// After prepare() from v: p = (b - H v) / d_f with d_f the frame's mean of
// diag(A^T Lambda A) + 1/sigma^2 (estimated by A^T Lambda A applied to ones).
msf_status feature(msf_plan *P, hipStream_t s)
{
    HIPCHK(launch_fill(P->p, P->nvox_total, 1.0f, s));
    HIPCHK(launch_forward(*P, PM_WEIGHTED, P->p, nullptr, P->sz, false, s));
    HIPCHK(launch_back(*P, P->sz, P->bp, false, s));
    HIPCHK(launch_vol_sum_bp(*P, s));
    HIPCHK(launch_scalar_reduce(*P, RW_DIAG, s));
    HIPCHK(launch_scale_feature(*P, s));
    return MSF_OK;
}

// Iterative refinement.  The iterate is x64 (FP64); the FP32 vector x holds
// the correction that the CG steps since the last refinement have built.
// Each refinement adds that correction to x64 and zeroes x, computes
// r = b - H x64 with the FP64 operator (exact.hip), and restarts every
// frame's CG from it (p = r), so the following FP32 steps solve for the next
// correction.  A frame is then active unless that residual meets the final
// tolerance or its steps are used up.  (Keeping the old direction across a
// replacement of the residual diverges on the stiff systems this is for: the
// FP32 and FP64 operators differ too much relative to the late residuals.)
// first: x64 = x (the start) instead of a fold.
msf_status refine_residual(msf_plan *P, bool first, hipStream_t s)
{
    if (!P->z64) {
        int64_t bytes = 0;
        hipError_t e = dalloc(&P->z64, (size_t)std::max<int64_t>(P->nmeas_total, 1), bytes);
        if (e == hipSuccess) e = dalloc(&P->x64, (size_t)std::max<int64_t>(P->nvox_total, 1), bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc refinement workspace");
        P->workspace_bytes += bytes;
    }
    if (first) HIPCHK(launch_fill_d(P->x64, P->nvox_total, s));
    HIPCHK(launch_fold_correction(*P, s));
    HIPCHK(launch_exact_data_residual(*P, P->x64, P->z64, s));
    HIPCHK(launch_vol_residual64(*P, s));
    HIPCHK(launch_scalar_reduce(*P, RW_REPLACE, s));
    return MSF_OK;
}

}  // namespace

msf_status msf_prox_features(msf_plan *P, const float *v, const float *y, const float *lam, double sigma, float *g_out,
                             void *stream)
{
    g_err.clear();
    if (!P || !v || !y || !lam || !g_out) { set_error("null argument"); return MSF_EINVAL; }
    if (!finite_pos(sigma)) { set_error("sigma must be positive and finite"); return MSF_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    msf_status st = prepare(P, v, y, lam, sigma, 0.0, 0, nullptr, s);
    if (st != MSF_OK) return st;
    if ((st = feature(P, s)) != MSF_OK) return st;
    HIPCHK(vol_to_public(*P, P->p, g_out, s));
    HIPCHK(hipStreamSynchronize(s));
    return MSF_OK;
}

msf_status msf_prox_solve(msf_plan *P, const float *v, const float *y, const float *lam, double sigma,
                          const msf_solve_opts *opts_in, float *x_out, msf_solve_stats *stats, void *stream)
{
    g_err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (!P || !v || !y || !lam || !x_out) { set_error("null argument"); return MSF_EINVAL; }
    if (!finite_pos(sigma)) { set_error("sigma must be positive and finite"); return MSF_EINVAL; }
    msf_solve_opts o;
    if (opts_in) o = *opts_in;
    else msf_solve_opts_default(&o);
    if (!(std::isfinite(o.tol) && o.tol >= 0.0) || o.max_iter < 0 || o.check_every < 1 || o.refine_every < 0) {
        set_error("invalid solver options (tol >= 0, max_iter >= 0, check_every >= 1, refine_every >= 0)");
        return MSF_EINVAL;
    }
    if (o.x0_mode == MSF_X0_USER && !o.x0) { set_error("x0_mode USER needs x0"); return MSF_EINVAL; }
    if (o.x0_mode == MSF_X0_CNN && (!o.cnn || cnn_kind(o.cnn) != MSF_CNN_WARM_START)) {
        set_error("x0_mode CNN needs a warm-start network (msf_cnn_create)");
        return MSF_EINVAL;
    }
    if (o.x0_mode != MSF_X0_V && o.x0_mode != MSF_X0_USER && o.x0_mode != MSF_X0_CNN) {
        set_error("unknown x0_mode"); return MSF_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int nf = P->nf;
    // With refinement the FP32 steps of each correction run to a tenth of tol
    // on their recursive residual; the FP64 residual decides at tol.
    const bool refine = o.refine_every > 0;
    msf_status pst = prepare(P, v, y, lam, sigma, refine ? 0.1 * o.tol : o.tol, o.max_iter,
                             o.x0_mode == MSF_X0_USER ? o.x0 : nullptr, s, o.tol);
    if (pst != MSF_OK) return pst;
    int32_t *hflags = (int32_t *)((double *)P->host_stage + 4);

    if (o.x0_mode == MSF_X0_CNN) {
        // learned start x_cnn = v + c f(v / c, g / c); kept per frame only if
        // finite and with a smaller residual than v (else the frame starts at v)
        msf_cnn *C = const_cast<msf_cnn *>(o.cnn);
        msf_status fs = feature(P, s);
        if (fs != MSF_OK) return fs;
        float *gpub = nullptr, *xpub = nullptr;
        HIPCHK(cnn_io_buffers(C, P->nvox_total, &gpub, &xpub));
        HIPCHK(vol_to_public(*P, P->p, gpub, s));
        HIPCHK(cnn_infer_internal(C, v, gpub, P->nf, P->nz, P->ny, P->nx, xpub, s));
        HIPCHK(vol_to_internal(*P, xpub, P->x, 0, nullptr, s));
        HIPCHK(launch_forward(*P, PM_RESID, P->x, P->sy, P->sz, false, s));
        HIPCHK(launch_back(*P, P->sz, P->bp, false, s));
        HIPCHK(launch_vol_residual_p(*P, s));
        HIPCHK(launch_scalar_reduce(*P, RW_CNN, s));
        HIPCHK(launch_vol_select(*P, s));
    }
    std::vector<double> rel0;
    if (stats && stats->start_rel_residual) {
        msf_status rs = start_residual(P, rel0, s);
        if (rs != MSF_OK) return rs;
    }

    // CG steps: one captured graph holds a whole check period (check_every
    // steps of six launches each); a shorter last period runs eagerly.
    const int period = o.check_every;
    if (P->timing && (int)P->ev.size() < 4 * period) {
        const size_t have = P->ev.size();
        P->ev.resize(4 * period, nullptr);
        for (size_t k = have; k < P->ev.size(); ++k) HIPCHK(hipEventCreate(&P->ev[k]));
    }
    bool use_graph = o.use_graph != 0;
    if (use_graph && (!P->graph_valid || P->graph_steps != period || P->graph_timing != P->timing)) {
        if (P->graph) (void)hipGraphExecDestroy(P->graph);
        P->graph = nullptr;
        P->graph_valid = false;
        hipStream_t cs;
        HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = hipSuccess;
            for (int k = 0; k < period && e2 == hipSuccess; ++k)
                e2 = launch_cg_step(*P, cs, P->timing ? &P->ev[4 * k] : nullptr);
            e = hipStreamEndCapture(cs, &graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&P->graph, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            if (!P->timing) return hip_fail(e, "CG step graph capture");
            (void)hipGetLastError();   // timed steps fall back to eager launches
            use_graph = false;
        } else {
            P->graph_valid = true;
            P->graph_steps = period;
            P->graph_timing = P->timing;
        }
    }
    int32_t *hact = hflags;
    int steps = 0;
    std::vector<float> step_fwd_ms, step_back_ms;
    auto fetch_active = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(hact, P->iscal + IS_ACTIVE * nf, sizeof(int32_t) * nf, hipMemcpyDeviceToHost,
                                      s);
        return e == hipSuccess ? hipStreamSynchronize(s) : e;
    };
    const int refine_period = refine ? ((o.refine_every + period - 1) / period) * period : 0;
    int since_refine = 0;
    if (refine) {
        // the start becomes the FP64 iterate; its residual with the FP64 operator
        msf_status rs = refine_residual(P, true, s);
        if (rs != MSF_OK) return rs;
    }
    HIPCHK(fetch_active());
    bool any = std::any_of(hact, hact + nf, [](int32_t a) { return a != 0; });
    while (steps < o.max_iter) {
        if (!any) {
            if (!refine || since_refine == 0) break;
            // every frame met tol on its recursive residual: confirm with the FP64 one
            msf_status rs = refine_residual(P, false, s);
            if (rs != MSF_OK) return rs;
            since_refine = 0;
            HIPCHK(fetch_active());
            any = std::any_of(hact, hact + nf, [](int32_t a) { return a != 0; });
            continue;
        }
        const int n = std::min(period, o.max_iter - steps);
        if (use_graph && n == period) {
            HIPCHK(hipGraphLaunch(P->graph, s));
        } else {
            for (int k = 0; k < n; ++k) HIPCHK(launch_cg_step(*P, s, P->timing ? &P->ev[4 * k] : nullptr));
        }
        steps += n;
        since_refine += n;
        if (refine && since_refine >= refine_period && steps < o.max_iter) {
            msf_status rs = refine_residual(P, false, s);
            if (rs != MSF_OK) return rs;
            since_refine = 0;
        }
        HIPCHK(fetch_active());
        if (P->timing) {
            for (int k = 0; k < n; ++k) {
                float a = 0.0f, b = 0.0f;
                HIPCHK(hipEventElapsedTime(&a, P->ev[4 * k], P->ev[4 * k + 1]));
                HIPCHK(hipEventElapsedTime(&b, P->ev[4 * k + 2], P->ev[4 * k + 3]));
                step_fwd_ms.push_back(a);
                step_back_ms.push_back(b);
            }
        }
        any = std::any_of(hact, hact + nf, [](int32_t a) { return a != 0; });
    }

    if (refine) {
        // steps since the last refinement (max_iter reached): fold them in and
        // report the FP64 residual of the final iterate; then x = x64 in FP32
        if (since_refine > 0) {
            HIPCHK(launch_fold_correction(*P, s));
            HIPCHK(launch_exact_data_residual(*P, P->x64, P->z64, s));
            HIPCHK(launch_vol_residual64(*P, s));
            HIPCHK(launch_scalar_reduce(*P, RW_TRUE, s));
        }
        HIPCHK(launch_d2f(P->x64, P->x, P->nvox_total, s));
    }
    HIPCHK(vol_to_public(*P, P->x, x_out, s));
    if (o.true_residual && !refine) {
        HIPCHK(launch_forward(*P, PM_RESID, P->x, P->sy, P->sz, false, s));
        HIPCHK(launch_back(*P, P->sz, P->bp, false, s));
        HIPCHK(launch_vol_true_residual(*P, s));
        HIPCHK(launch_scalar_reduce(*P, RW_TRUE, s));
    }
    double *hs = (double *)P->host_stage;
    int32_t *hi = (int32_t *)(hs + SC_COUNT * nf);
    HIPCHK(hipMemcpyAsync(hs, P->scal, sizeof(double) * SC_COUNT * nf, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hi, P->iscal, sizeof(int32_t) * IS_COUNT * nf, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));

    msf_status st = MSF_OK;
    for (int f = 0; f < nf; ++f) {
        const double rel = hs[SC_REL * nf + f];
        // refined solves are judged by their final FP64 residual
        const double judged = refine ? hs[SC_TRUE * nf + f] : rel;
        const bool conv = hs[SC_BNORM * nf + f] > 0.0 ? judged <= o.tol : hs[SC_GAMMA * nf + f] == 0.0;
        if (hi[IS_STATUS * nf + f] == MSF_EBREAKDOWN) st = MSF_EBREAKDOWN;
        else if (!conv && st == MSF_OK) st = MSF_NOT_CONVERGED;
        if (stats) {
            if (stats->iters) stats->iters[f] = hi[IS_ITERS * nf + f];
            if (stats->rel_residual) stats->rel_residual[f] = rel;
            if (stats->true_rel_residual)
                stats->true_rel_residual[f] = (o.true_residual || refine) ? hs[SC_TRUE * nf + f] : -1.0;
            if (stats->converged) stats->converged[f] = conv ? 1 : 0;
            if (stats->cnn_used) stats->cnn_used[f] = o.x0_mode == MSF_X0_CNN ? (uint8_t)hi[IS_CNN * nf + f] : 0;
            if (stats->start_rel_residual) stats->start_rel_residual[f] = rel0[f];
        }
    }
    if (P->timing && !step_fwd_ms.empty()) {
        // only steps in which every frame was still iterating: each such launch did the full batch
        int full = o.max_iter;
        for (int f = 0; f < nf; ++f) full = std::min(full, (int)hi[IS_ITERS * nf + f]);
        for (int k = 0; k < full && k < (int)step_fwd_ms.size(); ++k) {
            P->t_fwd_ms += step_fwd_ms[k];
            P->t_back_ms += step_back_ms[k];
            P->n_fwd++;
            P->n_back++;
        }
    }
    if (st == MSF_OK && o.x0_mode == MSF_X0_CNN)
        for (int f = 0; f < nf; ++f)
            if (!hi[IS_CNN * nf + f]) st = MSF_CNN_FALLBACK;
    if (st == MSF_EBREAKDOWN) set_error("CG breakdown: <p, H p> <= 0 or non-finite on some frame");
    if (stats) {
        stats->steps = steps;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

}  // extern "C"
