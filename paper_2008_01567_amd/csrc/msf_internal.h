// Internal declarations of libmsf (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/msf.h"

// ---------------------------------------------------------------------------
// Internal layouts (chosen for the circular orbit about the z axis):
//   volume   [frame][ny][nx][nz]   z fastest: all rays of one detector column
//            (fixed u, varying v) share one xy path, and a 64-lane wave of
//            consecutive detector rows reads consecutive z of one voxel column.
//   sinogram [view][nu][nv]        v fastest: a wave's rows are contiguous.
// The public layouts ([frame][nz][ny][nx], [view][nv][nu]) are converted at
// the API boundary by a tiled transpose.
// ---------------------------------------------------------------------------

enum ProjMode : int {
    PM_PLAIN = 0,     // out = A p
    PM_WEIGHTED = 1,  // out = Lambda (A p), partial += <A p, Lambda A p>
    PM_RESID = 2,     // out = Lambda (y - A p)
    PM_COUNT = 3,     // out = number of ray-voxel pieces of each ray (nnz of its row of A)
};

// Everything a projector launch needs (passed by value as a kernel argument).
// One detector column's piece of the xy line inside one xy cell (the voxel-
// driven adjoint's table): s range [fa, fb], the smaller and larger of the
// detector rows per unit z at the piece's two ends (rmin, rmax: they bound the
// rows through a voxel), the column's source offset sf and its index iu.
struct CellEntry {
    float fa, fb, rmin, rmax;
    double sf;
    int32_t iu, pad;
};

// The forward walk of one detector column's xy line, precomputed (back_mode
// 2): the cells it visits in order, as (iy * nx + ix, parameter where the
// line leaves the cell), after a head (number of cells, entry parameter).
struct WalkEntry {
    int32_t cell;
    float snext;
};
struct WalkHead {
    int32_t n;
    float s_in;
};

struct ProjParams {
    int nx, ny, nz, nu, nv, nf;
    double du, dv, rs, rsd, offu, offv;
    const double2 *cs;           // [n_views] (cos t, sin t)
    const int64_t *view_offset;  // [nf + 1]
    const int64_t *tile_offset;  // [nf + 1] projector tiles per frame (prefix)
    const int32_t *active;       // [nf] or nullptr (all active)
    int n_ug;                    // u-groups per view (columns / waves_per_group)
    int n_vc;                    // row chunks per column
    int rows_per_chunk;          // 64 * rays_per_lane
    int iv_lo, iv_hi;            // detector rows that can meet the volume
    int multi_row;               // a ray may meet one voxel within one xy piece in three or more rows
    int xcd_remap;
    int64_t nvox;                // voxels per frame
    int64_t total_tiles;
    const double2 *rzp;          // [nv] (height zp of detector row v, 1/zp; 1e290 when zp = 0)
    const double *imtab;         // [nu][nv] lxy(u) / zp(v) (lxy = xy distance source -> pixel; 1e290 lxy when zp = 0)
    const int32_t *cell_hdr;     // [n_views][ny * nx] number of columns meeting the cell (back_mode 2), or null
    const struct CellEntry *cell_ent;   // [n_views][ny * nx][cell_k], the first cell_hdr[] entries valid
    int cell_k;
    const struct WalkHead *walk_head;   // [n_views * nu] (back_mode 2), or null
    const struct WalkEntry *walk_ent;   // [n_views * nu][walk_stride]
    int walk_stride;                    // nx + ny + 2 (the walk's bound)
    // voxel-driven backprojector
    const struct ColEntry *cols; // [n_views * nu] column table
    int64_t g_tiles_per_frame;
    int g_zpl;                   // z voxels per lane
    const float *scale;          // [nu][nv] 3D ray length per unit of xy length: sqrt(1 + (zp / lxy)^2)
};

// The sinogram a backprojector reads is pre-multiplied by the ray's 3D length
// factor (the scale table), so the adjoint kernels never recompute it.

// One detector column's xy line (shared by all its rows), as the forward
// projector computes it; the voxel-driven backprojector reads it from a table
// so both use identical plane-crossing parameters.
struct ColEntry {
    double iex, iey, cx, cy;     // x/y plane k is crossed at s = k * iex + cx (resp. y)
    double sf, lxy, inv_lxy;     // source -> foot point, source -> pixel (xy), its inverse
    double s_in, s_out;          // xy-box clip
    int32_t hit, ixf, iyf, pad;  // hit flag; fixed cell index of an axis with zero direction component
};

// Per-frame scalars of the batched CG (device, FP64).
enum ScalarSlot : int {
    SC_GAMMA = 0,   // ||r||^2
    SC_PP,          // ||p||^2
    SC_PQ,          // <p, H p>
    SC_ALPHA,
    SC_BETA,
    SC_BNORM,       // ||b||
    SC_REL,         // ||r|| / ||b||
    SC_TRUE,        // true relative residual
    SC_DIAG,        // mean over voxels of diag(A^T Lambda A) (row-sum estimate) + 1/sigma^2
    SC_GCNN,        // ||b - H x_cnn||^2
    SC_COUNT
};
enum IScalarSlot : int { IS_ACTIVE = 0, IS_ITERS, IS_STATUS, IS_CNN, IS_COUNT };
// global solve constants live in consts[]: [0] = 1/sigma^2, [1] = tol of the recursive residual,
// [2] = max_iter, [3] = tol of the FP64 residual (refinement)

struct msf_plan {
    // geometry (host copy)
    int nx = 0, ny = 0, nz = 0, nf = 0, nu = 0, nv = 0;
    double du = 0, dv = 0, rs = 0, rsd = 0, offu = 0, offv = 0;
    std::vector<int64_t> view_offset;
    std::vector<double> angles;
    int64_t n_views = 0, nvox = 0, nvox_total = 0, nmeas_total = 0;
    int iv_lo = 0, iv_hi = -1;
    bool steep = false;                   // some ray may cross two z planes inside one xy cell
    bool multi_row = true;                // some ray may meet one voxel within one xy piece in 3+ rows
    msf_tiles tiles{};
    std::vector<int64_t> tile_offset;     // host copy of the projector tile prefix
    int64_t vol_blocks_per_frame = 0;     // blocks of the volume kernels per frame

    // device tables
    double2 *d_cs = nullptr;
    double2 *d_rzp = nullptr;             // [nv]
    double *d_imtab = nullptr;            // [nu][nv]
    int32_t *d_cell_hdr = nullptr;        // [n_views][ny * nx]   (built when back_mode 2 is first used)
    CellEntry *d_cell_ent = nullptr;      // [n_views][ny * nx][cell_k]
    WalkHead *d_walk_head = nullptr;      // [n_views * nu]               (built with the cell table)
    WalkEntry *d_walk_ent = nullptr;      // [n_views * nu][nx + ny + 2]
    int cell_k = 0;
    float *d_scale = nullptr;             // [nu][nv]
    double *part_g = nullptr;             // [nf * gather tiles per frame] ||r||^2 partials of the fused gather
    int64_t part_g_per_frame = 0;
    ColEntry *d_cols = nullptr;           // [n_views * nu]
    int64_t *d_view_offset = nullptr;
    int64_t *d_tile_offset = nullptr;

    // device workspace
    float *x = nullptr, *r = nullptr, *p = nullptr, *vin = nullptr;
    double *bp = nullptr;         // backprojection accumulator (FP64 atomic adds)
    double *z64 = nullptr;        // FP64 sinogram of the refinement residual (allocated on first use)
    double *x64 = nullptr;        // FP64 iterate of a refined solve (allocated with z64)
    float *sy = nullptr, *slam = nullptr, *sz = nullptr;
    double *part_proj = nullptr;  // [total_tiles]
    double *part_vol = nullptr;   // [nf * vol_blocks_per_frame]
    double *scal = nullptr;       // [SC_COUNT][nf]
    int32_t *iscal = nullptr;     // [IS_COUNT][nf]
    double *consts = nullptr;     // [4]
    int32_t *flags = nullptr;     // [4] validation counters
    void *host_stage = nullptr;   // pinned host staging
    size_t host_stage_bytes = 0;
    int64_t workspace_bytes = 0;

    // captured CG steps (one graph = graph_steps CG steps)
    hipGraphExec_t graph = nullptr;
    bool graph_valid = false;
    int graph_steps = 0;
    bool graph_timing = false;

    // live kernel timing with HIP events (msf_plan_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> ev;        // 4 per CG step of a check period
    double t_fwd_ms = 0.0, t_back_ms = 0.0;
    int64_t n_fwd = 0, n_back = 0;

    ProjParams proj_params(bool with_active) const;
    int64_t total_tiles() const { return tile_offset.empty() ? 0 : tile_offset.back(); }
};

// error reporting (thread-local message)
void set_error(const std::string &msg);
msf_status hip_fail(hipError_t e, const char *where);
// public <-> internal layouts (tiled transposes); check 1: count non-finite, 2: negative or non-finite, into *flag
hipError_t vol_to_internal(const msf_plan &P, const float *in, float *out, int check, int32_t *flag, hipStream_t s);
hipError_t vol_to_public(const msf_plan &P, const float *in, float *out, hipStream_t s);
hipError_t sino_to_internal(const msf_plan &P, const float *in, float *out, int check, int32_t *flag, hipStream_t s);
hipError_t sino_to_public(const msf_plan &P, const float *in, float *out, hipStream_t s);

// ------------------------------------------------------------ launchers --
hipError_t launch_forward(const msf_plan &P, int mode, const float *vol, const float *y, float *out,
                          bool with_active, hipStream_t s);
hipError_t launch_back_scatter(const msf_plan &P, const float *sino, double *vol_acc, bool with_active,
                               hipStream_t s);
hipError_t launch_back_gather(const msf_plan &P, const float *sino, double *vol_out, bool with_active,
                              hipStream_t s);
// A^T into the FP64 accumulator with the plan's back_mode (scatter adds into a
// zeroed buffer; gather overwrites every voxel of the frames it processes)
hipError_t launch_back(const msf_plan &P, const float *sino, double *vol, bool with_active, hipStream_t s);
// voxel-driven A^T fused with the CG update of x and r (partials of ||r||^2 in part_g)
hipError_t launch_back_gather_update(const msf_plan &P, hipStream_t s);
// per (view, xy cell) piece table of the voxel-driven adjoint (back_mode 2); overflow count in flags[4]
hipError_t launch_cell_table(msf_plan &P, hipStream_t s);
// per detector column walk table of the forward projector (back_mode 2)
hipError_t launch_walk_table(msf_plan &P, hipStream_t s);
// sino[i] *= scale[i mod (nu nv)] (internal layout)
hipError_t launch_prescale(const msf_plan &P, float *sino, hipStream_t s);
hipError_t launch_scale_table(msf_plan &P, hipStream_t s);
hipError_t launch_col_table(msf_plan &P, hipStream_t s);

// batched transpose [B][R][C] -> [B][C][R]; counts entries failing the check
// into flags[check_slot] (check: 0 none, 1 non-finite, 2 negative or non-finite)
hipError_t launch_transpose(const float *in, float *out, int64_t B, int R, int C, int check, int32_t *flags,
                            hipStream_t s);

// CG vector / scalar kernels (see cg.hip)
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_d(double *p, int64_t n, hipStream_t s);
hipError_t launch_d2f(const double *src, float *dst, int64_t n, hipStream_t s);
hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t s);
hipError_t launch_sino_mul(const float *a, const float *b, float *out, int64_t n, hipStream_t s);
// out = a * b * scale[i mod per_view]
hipError_t launch_sino_mul_scaled(const float *a, const float *b, const float *scale, int64_t per_view, float *out,
                                  int64_t n, hipStream_t s);
hipError_t launch_vol_bnorm(msf_plan &P, hipStream_t s);
hipError_t launch_vol_init_residual(msf_plan &P, hipStream_t s);
hipError_t launch_vol_true_residual(msf_plan &P, hipStream_t s);
hipError_t launch_scalar_reduce(msf_plan &P, int what, hipStream_t s);
// ev: 4 events (forward start/stop, backprojection start/stop) or nullptr
hipError_t launch_cg_step(msf_plan &P, hipStream_t s, hipEvent_t *ev);

enum ReduceWhat : int {
    RW_BNORM = 0,      // part_vol -> SC_BNORM
    RW_INIT = 1,       // part_vol -> SC_GAMMA, SC_PP = SC_GAMMA, active flags
    RW_TRUE = 2,       // part_vol -> SC_TRUE
    RW_DIAG = 3,       // part_vol (sum of A^T Lambda A 1) -> SC_DIAG
    RW_CNN = 4,        // part_vol -> SC_GCNN, then choose the start per frame (IS_CNN)
    RW_REPLACE = 5,    // part_vol of the FP64 residual (CG restarted from it) -> SC_GAMMA, SC_PP, SC_REL,
                       // SC_TRUE, active flags (iteration counts kept)
};
// bp = A^T Lambda (y - A x) with FP64 lengths, sinogram (z64) and sums, x an FP64 volume (exact.hip)
hipError_t launch_exact_data_residual(msf_plan &P, const double *x, double *z64, hipStream_t s);
// refinement: x64 += x (the FP32 correction), x = 0
hipError_t launch_fold_correction(msf_plan &P, hipStream_t s);
// refinement: r = p = bp + (v - x64) / sigma^2, partial ||r||^2 into part_vol; clears bp
hipError_t launch_vol_residual64(msf_plan &P, hipStream_t s);
hipError_t launch_vol_sum_bp(msf_plan &P, hipStream_t s);
// p = r / diag_f (the network's residual feature, internal layout)
hipError_t launch_scale_feature(msf_plan &P, hipStream_t s);
// r = b - H x into p only (the learned start's residual), partial ||.||^2
hipError_t launch_vol_residual_p(msf_plan &P, hipStream_t s);
// per frame: keep the learned start (r = p) or go back to v (x = v, p = r)
hipError_t launch_vol_select(msf_plan &P, hipStream_t s);
// network evaluation (cnn.hip): x0 = v + c f(v / c, g / c) on public-layout volumes
hipError_t cnn_infer_internal(struct msf_cnn *C, const float *v, const float *g, int N, int Z, int Y, int X, float *x0,
                              hipStream_t s);
// MSF_CNN_WARM_START or MSF_CNN_DENOISER
int cnn_kind(const struct msf_cnn *C);
// the 2.5D denoiser in plane 1 (xy), 2 (yz) or 3 (zx) of a [T][Z][Y][X]
// sequence; out must not overlap w; planes 2 and 3 use two scratch volumes
hipError_t denoise25_internal(struct msf_cnn *C, const float *w, int T, int Z, int Y, int X, int plane, float *out,
                              float *scratch_a, float *scratch_b, hipStream_t s);
