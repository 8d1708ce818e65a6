// Cone-beam forward projector A and its adjoint A^T for gfx950.
//
// A[i][j] is the length of ray i (point source -> detector pixel centre)
// inside voxel j (paper Sec. II: the system matrix of eq. (2);
// the exact ray-voxel length is this library's discretisation of it).  The
// lengths are computed on the fly by a Siddon-type traversal (Siddon 1985):
// the ray is cut at every voxel-plane crossing and each piece is credited to
// the voxel it lies in.
//
// Mapping to the hardware.  The orbit is circular about z, so every ray of one
// detector column (fixed u, all rows v) has the same projection onto the xy
// plane.  One 64-lane wave owns one column: the 2D walk through the xy cells
// of that line is uniform across the wave (no divergence), and each lane
// follows the z coordinate of its own rows (rays_per_lane rows, 64 apart),
// splitting a cell's piece where its ray crosses a z plane.  With the internal
// z-fastest volume layout the lanes of a wave read consecutive z of one voxel
// column: coalesced loads from L2 / the Infinity Cache.  There is no dense
// contraction here, so no MFMA.
//
// Precision.  Plane-crossing parameters are computed in FP64 from plane
// indices (never accumulated), then rounded to FP32; piece lengths are FP32
// differences of consecutive rounded parameters, so they telescope exactly
// along a ray.  The xy path is parametrised by s, the xy distance from the
// line's closest approach to the rotation axis (|s| <= half the volume
// diagonal), which keeps FP32 parameters small.
//
// A piece's 3D length is its xy length times sqrt(1 + (zp / lxy)^2), a factor
// of the ray alone (detector column u and row v; the same for every view):
// the forward applies it to the finished ray sum from a [nu][nv] table, and
// the adjoints read sinograms that are already multiplied by it.
//
// The adjoint comes in two forms that use bit-identical lengths.  The scatter
// runs the very same traversal and adds length * value into each voxel with
// hardware FP64 atomics (an FP64 accumulator keeps the mixed-sign sums of CG
// free of FP32 cancellation).  The gather (the default) is voxel-driven,
// deterministic and atomic-free; it recomputes each piece with the forward
// walk's crossing expressions.
#include "msf_internal.h"

#include <cmath>

namespace {

constexpr int WAVE = 64;
constexpr int FLUSH = 16;   // cells per FP32 partial sum before it is added to the FP64 ray sum

// Raw buffer loads of element idx of a row of n elements (a table row, a
// sinogram column, a voxel column): 32-bit offsets from a scalar base, and the
// hardware range check returns 0 for idx outside [0, n).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ float row_f32(__amdgpu_buffer_rsrc_t r, int idx)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4, 0, 0));
}
__device__ __forceinline__ double row_f64(__amdgpu_buffer_rsrc_t r, int idx)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8, 0, 0));
}
// element idx + 1: the constant goes into the instruction's offset field,
// which the range check includes (reads past the row still give 0)
__device__ __forceinline__ float row_f32_next(__amdgpu_buffer_rsrc_t r, int idx)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4 + 4, 0, 0));
}
__device__ __forceinline__ double row_f64_next(__amdgpu_buffer_rsrc_t r, int idx)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8 + 8, 0, 0));
}

// Parameter of the crossing with plane k of an axis: s = k * inv + c0, with
// inv = 1/e (direction component) and c0 = (-half - f) * inv.  Every kernel
// computes crossings with this one expression, so A and A^T see the same
// rounded values.
__device__ __forceinline__ double plane_s(int k, double inv, double c0) { return fma((double)k, inv, c0); }

struct Column {
    double iex, iey;    // 1/ex, 1/ey (0 when the component is 0)
    double cx, cy;      // crossing offsets (see plane_s)
    double sf;          // xy distance source -> foot point (the source sits at s = -sf)
    double lxy;         // xy distance source -> pixel
    double inv_lxy;
    double s_in, s_out; // xy-box clip of the line
    int ix, iy;         // entry cell
    int stepx, stepy;
    double sxn, syn;    // next x / y plane crossing
};

// Axis helper: range of s inside [0, n] planes, or false if the line misses.
__device__ __forceinline__ bool axis_range(double e, double f, double h, int n, double &inv, double &c0,
                                           double &s0, double &s1)
{
    if (e != 0.0) {
        inv = 1.0 / e;
        c0 = (-h - f) * inv;
        const double a = plane_s(0, inv, c0), b = plane_s(n, inv, c0);
        s0 = fmin(a, b);
        s1 = fmax(a, b);
        return true;
    }
    inv = 0.0;
    c0 = 0.0;
    if (!(f >= -h && f < h)) return false;
    s0 = -INFINITY;
    s1 = INFINITY;
    return true;
}

__device__ __forceinline__ bool column_setup(const ProjParams &P, int view, int iu, Column &c)
{
    const double2 cs = P.cs[view];
    const double u = (iu - 0.5 * (P.nu - 1)) * P.du + P.offu;
    const double sx = P.rs * cs.x, sy = P.rs * cs.y;
    const double dx = -P.rsd * cs.x - u * cs.y;
    const double dy = -P.rsd * cs.y + u * cs.x;
    c.lxy = sqrt(dx * dx + dy * dy);
    const double ex = dx / c.lxy, ey = dy / c.lxy;
    c.inv_lxy = 1.0 / c.lxy;
    c.sf = -(sx * ex + sy * ey);
    const double fx = sx + c.sf * ex, fy = sy + c.sf * ey;
    const double hx = 0.5 * P.nx, hy = 0.5 * P.ny;
    double sx0, sx1, sy0, sy1;
    if (!axis_range(ex, fx, hx, P.nx, c.iex, c.cx, sx0, sx1)) return false;
    if (!axis_range(ey, fy, hy, P.ny, c.iey, c.cy, sy0, sy1)) return false;
    c.s_in = fmax(sx0, sy0);
    c.s_out = fmin(sx1, sy1);
    if (!(c.s_out > c.s_in)) return false;
    c.stepx = ex > 0.0 ? 1 : (ex < 0.0 ? -1 : 0);
    c.stepy = ey > 0.0 ? 1 : (ey < 0.0 ? -1 : 0);
    // entry cell: the entering axis from the direction, the other from the entry point
    if (sx0 >= sy0) c.ix = c.stepx > 0 ? 0 : P.nx - 1;
    else c.ix = min(max((int)floor(fx + ex * c.s_in + hx), 0), P.nx - 1);
    if (sy0 >= sx0) c.iy = c.stepy > 0 ? 0 : P.ny - 1;
    else c.iy = min(max((int)floor(fy + ey * c.s_in + hy), 0), P.ny - 1);
    c.sxn = c.stepx ? plane_s(c.ix + (c.stepx > 0), c.iex, c.cx) : INFINITY;
    c.syn = c.stepy ? plane_s(c.iy + (c.stepy > 0), c.iey, c.cy) : INFINITY;
    return true;
}

// The walk is the same for the whole wave: keep its indices in scalar registers.
__device__ __forceinline__ void make_uniform(Column &c)
{
    c.ix = __builtin_amdgcn_readfirstlane(c.ix);
    c.iy = __builtin_amdgcn_readfirstlane(c.iy);
    c.stepx = __builtin_amdgcn_readfirstlane(c.stepx);
    c.stepy = __builtin_amdgcn_readfirstlane(c.stepy);
}

// The ray of height zp on the detector (xy length lxy) is at height
// z = zp (s + sf) / lxy; it crosses z plane k (z = k - nz/2) at
//     s = (k - nz/2) * im - sf,   im = lxy / zp,
// evaluated as fma(k - nz/2, im, -sf) by every kernel.
__device__ __forceinline__ double zplane_s(int k, double hz, double im, double sf)
{
    return fma((double)k - hz, im, -sf);
}

// z-state of one ray (one detector row) along the shared xy line.
struct RayZ {
    double im, sf;      // see zplane_s
    float lzi, lzo;     // s-range inside the z slab of the volume
    float szn;          // next z-plane crossing
    int iz, zstep;
    // open walk: kd = index of the next plane minus nz/2 (an exact double),
    // nsf = -sf (+inf for a ray that crosses no plane, so szn stays +inf), the
    // voxel's byte offset in the column and its step, and the high word of
    // the step as a double (the low word of +-1.0 is 0)
    double kd, nsf;
    int izb, zstepb, zsd_hi;
};

// OPEN: the ray's z slab index is not clamped to the volume.  Outside [0, nz)
// it addresses no voxel (the loads of the open walk return 0 there), so the
// walk needs no clipping of the pieces to the volume's z faces: it crosses the
// face planes like any other plane, at the same rounded parameters.
template <bool OPEN = false>
__device__ __forceinline__ void ray_setup(const ProjParams &P, const Column &c, int iu, int iv, bool valid, RayZ &z)
{
    const double hz = 0.5 * P.nz;
    const double2 zr = P.rzp[min(iv, P.nv - 1)];
    const double zp = zr.x;
    z.sf = c.sf;
    double lzi, lzo;
    const double z_in = zp * (c.s_in + c.sf) * c.inv_lxy;   // height where the line enters the xy box
    if (zp != 0.0) {
        z.im = P.imtab[(int64_t)iu * P.nv + min(iv, P.nv - 1)];
        const double a = zplane_s(0, hz, z.im, c.sf), b = zplane_s(P.nz, hz, z.im, c.sf);
        lzi = fmin(a, b);
        lzo = fmax(a, b);
    } else {
        z.im = 0.0;
        const bool in = z_in >= -hz && z_in < hz;
        lzi = in ? -INFINITY : INFINITY;
        lzo = in ? INFINITY : -INFINITY;
    }
    z.zstep = zp > 0.0 ? 1 : (zp < 0.0 ? -1 : 0);
    const double start = fmax(c.s_in, lzi);
    if (!valid || !(fmin(c.s_out, lzo) > start)) {
        z.lzi = INFINITY;
        z.lzo = -INFINITY;
        z.iz = OPEN ? -(1 << 24) : 0;   // open walk: far outside, never crossing back in
        z.szn = INFINITY;
        if (OPEN) {
            z.zstep = 0;
            z.izb = z.iz * 4;
            z.zstepb = 0;
            z.zsd_hi = 0;
            z.kd = 0.0;
            z.nsf = INFINITY;
        }
        return;
    }
    z.lzi = (float)lzi;
    z.lzo = (float)lzo;
    if (OPEN) z.iz = (int)floor(z_in + hz);
    else if (lzi >= c.s_in) z.iz = z.zstep > 0 ? 0 : P.nz - 1;
    else z.iz = min(max((int)floor(z_in + hz), 0), P.nz - 1);
    z.szn = z.zstep ? (float)zplane_s(z.iz + (z.zstep > 0), hz, z.im, z.sf) : INFINITY;
    if (OPEN) {
        z.izb = z.iz * 4;
        z.zstepb = z.zstep * 4;
        z.zsd_hi = z.zstep > 0 ? 0x3FF00000 : (z.zstep < 0 ? (int)0xBFF00000u : 0);
        z.kd = (double)(z.iz + (z.zstep > 0)) - hz;   // exact: an integer or half-integer
        z.nsf = z.zstep ? -z.sf : INFINITY;            // then fma(kd, im, nsf) is szn
    }
}

// One ray inside the xy cell [scur, snext] when at most one z plane can be
// crossed per cell (|dz/ds| * sqrt(2) < 1, checked at plan creation): the
// piece splits into (iz, l1) and (iz2, l2), l2 = 0 without a crossing.
struct Pieces {
    int iz, iz2;
    float l1, l2;
    bool cross;
};

__device__ __forceinline__ Pieces ray_pieces(const RayZ &z, float scur, float snext, int nz)
{
    Pieces q;
    const float a = fmaxf(scur, z.lzi);
    const float b = fminf(snext, z.lzo);
    const bool on = b > a;
    q.cross = on && z.szn < b;
    const float mid = q.cross ? fmaxf(z.szn, a) : b;
    q.l1 = on ? mid - a : 0.0f;
    q.l2 = q.cross ? b - mid : 0.0f;
    q.iz = z.iz;
    q.iz2 = min(max(z.iz + (q.cross ? z.zstep : 0), 0), nz - 1);
    return q;
}

__device__ __forceinline__ void ray_advance(RayZ &z, const Pieces &q, double hz)
{
    // branch-free: iz2 == iz without a crossing
    const float nxt = (float)zplane_s(q.iz2 + (z.zstep > 0), hz, z.im, z.sf);
    z.szn = q.cross ? nxt : z.szn;
    z.iz = q.iz2;
}

// Open walk (see ray_setup<true>): the pieces of the cell [scur, snext] on
// both sides of at most one z crossing, with no clipping to the volume; the
// voxels as byte offsets in the column.
struct PiecesOpen {
    int ob1, ob2;
    float l1, l2;
    bool cross;
};

__device__ __forceinline__ PiecesOpen ray_pieces_open(const RayZ &z, float scur, float snext)
{
    PiecesOpen q;
    q.cross = z.szn < snext;
    // cross ? max(szn, scur) : snext, as one median (scur <= snext along the walk)
    const float mid = __builtin_amdgcn_fmed3f(z.szn, scur, snext);
    q.l1 = mid - scur;
    q.l2 = snext - mid;     // exactly 0 without a crossing (mid = snext)
    q.ob1 = z.izb;
    q.ob2 = z.izb + (q.cross ? z.zstepb : 0);
    return q;
}

// After a crossing the next plane is one step on; szn is recomputed from kd
// either way (without a crossing that gives the same value), with the same
// rounded expression as zplane_s since kd equals (double)k - nz/2 exactly.
__device__ __forceinline__ void ray_advance_open(RayZ &z, const PiecesOpen &q)
{
    z.kd += __hiloint2double(q.cross ? z.zsd_hi : 0, 0);
    z.szn = (float)fma(z.kd, z.im, z.nsf);
    z.izb = q.ob2;
}

// General case (steep rays): walk every z crossing inside the cell.
template <class Op>
__device__ __forceinline__ void ray_cell_general(RayZ &z, float scur, float snext, int nz, Op &&op)
{
    const double hz = 0.5 * nz;
    const float a = fmaxf(scur, z.lzi);
    const float b = fminf(snext, z.lzo);
    if (!(b > a)) return;
    float sa = a;
    while (z.szn < b) {
        const float l = z.szn - sa;
        if (l > 0.0f) op(z.iz, l);
        sa = fmaxf(sa, z.szn);
        z.iz += z.zstep;
        if ((unsigned)z.iz >= (unsigned)nz) {   // left the volume through a z face
            z.lzo = -INFINITY;
            return;
        }
        z.szn = (float)zplane_s(z.iz + (z.zstep > 0), hz, z.im, z.sf);
    }
    op(z.iz, b - sa);
}

__device__ __forceinline__ int64_t logical_tile(int64_t b, int64_t G, int remap)
{
    // Workgroups are dispatched round-robin over the 8 XCDs (b mod 8).  The
    // remap gives each XCD one contiguous range of the tile list, so the tiles
    // of a frame (and of one z-chunk of it) share that XCD's L2.
    if (!remap) return b;
    const int64_t xcd = b & 7, idx = b >> 3;
    const int64_t per = G >> 3, rem = G & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

__device__ __forceinline__ int frame_of_tile(const int64_t *off, int nf, int64_t t)
{
    int lo = 0, hi = nf;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct Tile {
    int frame, view, iu, vc;
    bool ok;
};

__device__ __forceinline__ Tile decode_tile(const ProjParams &P, int64_t t, int wave, int nwaves)
{
    Tile T;
    T.frame = frame_of_tile(P.tile_offset, P.nf, t);
    const int64_t local = t - P.tile_offset[T.frame];
    const int vf = (int)(P.view_offset[T.frame + 1] - P.view_offset[T.frame]);
    const int64_t per_vc = (int64_t)vf * P.n_ug;
    T.vc = (int)(local / per_vc);
    const int rem = (int)(local - (int64_t)T.vc * per_vc);
    T.view = (int)P.view_offset[T.frame] + rem / P.n_ug;
    T.iu = (rem % P.n_ug) * nwaves + wave;
    T.ok = T.iu < P.nu && (P.active == nullptr || P.active[T.frame] != 0);
    return T;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Uniform 2D walk of the column's xy line; body(colp_offset, scur, snext)
// is called once per xy cell, then flush() every FLUSH cells.
template <class Body, class Flush>
__device__ __forceinline__ void walk_xy(const ProjParams &P, const Column &c, Body &&body, Flush &&flush)
{
    float scur = (float)c.s_in;
    int ix = c.ix, iy = c.iy;
    double sxn = c.sxn, syn = c.syn;
    int k = 0;
    for (int guard = P.nx + P.ny + 2; guard > 0; --guard) {
        const double s_next = fmin(fmin(sxn, syn), c.s_out);
        const float snext = (float)s_next;
        body((int64_t)(iy * P.nx + ix) * P.nz, scur, snext);
        if (++k == FLUSH) {
            flush();
            k = 0;
        }
        if (s_next >= c.s_out) break;
        if (sxn <= syn) {
            ix += c.stepx;
            if ((unsigned)ix >= (unsigned)P.nx) break;
            sxn = plane_s(ix + (c.stepx > 0), c.iex, c.cx);
        } else {
            iy += c.stepy;
            if ((unsigned)iy >= (unsigned)P.ny) break;
            syn = plane_s(iy + (c.stepy > 0), c.iey, c.cy);
        }
        scur = snext;
    }
    flush();
}

// The same walk read from the column's precomputed table (bit-identical
// cells and parameters); the entries of the next 8 cells are loaded while the
// current ones are processed.
//
// PAD: the body adds nothing for an empty cell [s, s] (every piece has length
// 0 and the walk state stays valid), so a block of 8 cells is processed
// whole, the cells past the end repeating the last one with zero length.
// With no branch between its cells a block is one straight run of code, and
// the loads of later cells can be issued before the sums of earlier ones.
// The flush still comes after every FLUSH (= 2 blocks) cells, as without PAD.
template <bool PAD = false, class Body, class Flush>
__device__ __forceinline__ void walk_table(const ProjParams &P, int64_t col, Body &&body, Flush &&flush)
{
    const WalkHead h = P.walk_head[col];
    const WalkEntry *e = P.walk_ent + col * P.walk_stride;
    constexpr int B = 8;
    static_assert(!PAD || FLUSH == 2 * B, "PAD flushes every second block");
    float scur = h.s_in;
    int k = 0;
    // PAD reads past the walk's end as its last entry; an empty walk runs no block
    const int last = PAD ? max(h.n - 1, 0) : P.walk_stride - 1;
    WalkEntry next[B];
#pragma unroll
    for (int j = 0; j < B; ++j) next[j] = e[min(j, last)];
    for (int c0 = 0; c0 < h.n; c0 += B) {
        WalkEntry cur[B];
#pragma unroll
        for (int j = 0; j < B; ++j) cur[j] = next[j];
        if (c0 + B < h.n) {
#pragma unroll
            for (int j = 0; j < B; ++j) next[j] = e[min(c0 + B + j, last)];
        }
        if (PAD) {
#pragma unroll
            for (int j = 0; j < B; ++j) {
                body((int64_t)cur[j].cell * P.nz, scur, cur[j].snext);
                scur = cur[j].snext;
            }
            if (c0 & B) flush();
        } else {
#pragma unroll
            for (int j = 0; j < B; ++j) {
                if (c0 + j >= h.n) break;
                body((int64_t)cur[j].cell * P.nz, scur, cur[j].snext);
                if (++k == FLUSH) {
                    flush();
                    k = 0;
                }
                scur = cur[j].snext;
            }
        }
    }
    flush();
}

// One thread per detector column: record the column's walk (the same walk_xy).
__global__ void k_walk_table(const ProjParams P, int64_t n_cols, WalkHead *__restrict__ head,
                             WalkEntry *__restrict__ ent)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_cols) return;
    Column c;
    WalkHead h{0, 0.0f};
    if (column_setup(P, (int)(i / P.nu), (int)(i % P.nu), c)) {
        h.s_in = (float)c.s_in;
        WalkEntry *e = ent + i * P.walk_stride;
        int n = 0;
        walk_xy(P, c, [&](int64_t off, float, float snext) {
            e[n].cell = (int32_t)(off / P.nz);
            e[n].snext = snext;
            ++n;
        }, [] {});
        h.n = n;
    }
    head[i] = h;
}

// Five rays per lane from the walk table fit in 96 registers without spilling,
// which runs 5 waves per SIMD instead of the 4 that 110 registers allow
// (256^3 x 24: 7.33 -> 7.13 ms per projection).  Six would spill.
template <int R, int MODE, bool STEEP, bool WT>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu((R == 5 && WT && (MODE == PM_PLAIN || MODE == PM_WEIGHTED)) ? 5 : 1)))
void k_forward(const ProjParams P, const float *__restrict__ vol,
                                                 const float *__restrict__ lam, const float *__restrict__ y,
                                                 float *__restrict__ out, double *__restrict__ partial)
{
    const int nwaves = blockDim.x / WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x % WAVE;
    const int64_t t = logical_tile(blockIdx.x, gridDim.x, P.xcd_remap);
    const Tile T = decode_tile(P, t, wave, nwaves);
    double part = 0.0;
    if (T.ok) {
        int iv[R];
        double acc[R];   // FP64 ray sums, fed by FP32 partial sums of FLUSH cells
        float acc32[R];
        RayZ z[R];
        Column c;
        const bool hit = column_setup(P, T.view, T.iu, c);
        make_uniform(c);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            iv[r] = P.iv_lo + T.vc * P.rows_per_chunk + r * WAVE + lane;
            acc[r] = 0.0;
            acc32[r] = 0.0f;
            if (hit) ray_setup<MODE != PM_COUNT && !STEEP>(P, c, T.iu, iv[r], iv[r] <= P.iv_hi, z[r]);
        }
        if (hit) {
            const float *volf = vol + (int64_t)T.frame * P.nvox;
            auto flush = [&]() {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    acc[r] += (double)acc32[r];
                    acc32[r] = 0.0f;
                }
            };
            auto cell_body = [&](int64_t off, float scur, float snext) {
                const float *colp = volf + off;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (MODE == PM_COUNT) {
                        if (STEEP) {
                            ray_cell_general(z[r], scur, snext, P.nz, [&](int, float l) { acc32[r] += l > 0.0f; });
                        } else {
                            const Pieces q = ray_pieces(z[r], scur, snext, P.nz);
                            acc32[r] += (float)(q.l1 > 0.0f) + (float)(q.l2 > 0.0f);
                            ray_advance(z[r], q, 0.5 * P.nz);
                        }
                    } else if (STEEP) {
                        ray_cell_general(z[r], scur, snext, P.nz,
                                         [&](int iz, float l) { acc32[r] = fmaf(l, colp[iz], acc32[r]); });
                    }
                }
                if (MODE != PM_COUNT && !STEEP) {
                    // all pieces first, then all 2R loads, then the sums: one wait per cell
                    PiecesOpen q[R];
                    float p1[R], p2[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) q[r] = ray_pieces_open(z[r], scur, snext);
                    // slabs outside [0, nz) read 0 (range-checked loads)
                    const __amdgpu_buffer_rsrc_t colr = row_rsrc(colp, P.nz * 4);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        p1[r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(colr, q[r].ob1, 0, 0));
                        p2[r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(colr, q[r].ob2, 0, 0));
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        acc32[r] = fmaf(q[r].l2, p2[r], fmaf(q[r].l1, p1[r], acc32[r]));
                        ray_advance_open(z[r], q[r]);
                    }
                }
            };
            if (WT) walk_table<MODE != PM_COUNT && !STEEP>(P, (int64_t)T.view * P.nu + T.iu, cell_body, flush);
            else walk_xy(P, c, cell_body, flush);
        }
        const int64_t base = (int64_t)T.view * P.nu * P.nv + (int64_t)T.iu * P.nv;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (iv[r] > P.iv_hi) continue;
            const int64_t idx = base + iv[r];
            const double sc = P.scale[(int64_t)T.iu * P.nv + iv[r]];
            const double w = hit ? acc[r] * (MODE == PM_COUNT ? 1.0 : sc) : 0.0;
            if (MODE == PM_PLAIN || MODE == PM_COUNT) {
                out[idx] = (float)w;
            } else if (MODE == PM_WEIGHTED) {
                // output pre-scaled for the adjoint: sc Lambda A p
                const double l = lam[idx];
                out[idx] = (float)(sc * l * w);
                part += w * l * w;
            } else {
                out[idx] = (float)(sc * (double)lam[idx] * ((double)y[idx] - w));
            }
        }
    }
    if (MODE == PM_WEIGHTED) {
        __shared__ double red[4];
        part = wave_sum(part);
        if (lane == 0) red[wave] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w) s += red[w];
            partial[t] = s;
        }
    }
}

template <int R, bool STEEP>
__global__ __launch_bounds__(256) void k_back_scatter(const ProjParams P, const float *__restrict__ sino,
                                                      double *__restrict__ vol)
{
    const int nwaves = blockDim.x / WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x % WAVE;
    const int64_t t = logical_tile(blockIdx.x, gridDim.x, P.xcd_remap);
    const Tile T = decode_tile(P, t, wave, nwaves);
    if (!T.ok) return;
    Column c;
    if (!column_setup(P, T.view, T.iu, c)) return;
    make_uniform(c);
    RayZ z[R];
    float val[R];
    const int64_t base = (int64_t)T.view * P.nu * P.nv + (int64_t)T.iu * P.nv;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iv = P.iv_lo + T.vc * P.rows_per_chunk + r * WAVE + lane;
        const bool valid = iv <= P.iv_hi;
        ray_setup(P, c, T.iu, iv, valid, z[r]);
        val[r] = valid ? sino[base + iv] : 0.0f;   // pre-scaled sinogram
        if (val[r] == 0.0f) {   // nothing to add: skip this ray's atomics
            z[r].lzi = INFINITY;
            z[r].lzo = -INFINITY;
        }
    }
    double *volf = vol + (int64_t)T.frame * P.nvox;
    walk_xy(P, c, [&](int64_t off, float scur, float snext) {
        double *colp = volf + off;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double v = val[r];
            if (STEEP) {
                ray_cell_general(z[r], scur, snext, P.nz,
                                 [&](int iz, float l) { unsafeAtomicAdd(colp + iz, (double)l * v); });
            } else {
                const Pieces q = ray_pieces(z[r], scur, snext, P.nz);
                if (q.l1 > 0.0f) unsafeAtomicAdd(colp + q.iz, (double)q.l1 * v);
                if (q.l2 > 0.0f) unsafeAtomicAdd(colp + q.iz2, (double)q.l2 * v);
                ray_advance(z[r], q, 0.5 * P.nz);
            }
        }
    }, [] {});
}


__global__ void k_col_table(const ProjParams P, int64_t n_views, ColEntry *__restrict__ tab)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_views * P.nu) return;
    Column c;
    const bool hit = column_setup(P, (int)(i / P.nu), (int)(i % P.nu), c);
    ColEntry e;
    e.iex = c.iex; e.iey = c.iey; e.cx = c.cx; e.cy = c.cy;
    e.sf = c.sf; e.lxy = c.lxy; e.inv_lxy = c.inv_lxy;
    e.s_in = c.s_in; e.s_out = c.s_out;
    e.hit = hit ? 1 : 0;
    e.ixf = hit ? c.ix : 0;
    e.iyf = hit ? c.iy : 0;
    e.pad = 0;
    tab[i] = e;
}

// Voxel-driven A^T.  One wave owns 64 * ZPL consecutive z voxels of one voxel
// column (ix, iy) of one frame and loops over that frame's views.  For each
// view the detector columns whose xy line meets the cell come from the
// projections of the cell's four corners; for each of them (uniform) the
// cell's piece [a, b] of the line uses the forward walk's crossing
// expressions, and each lane finds the detector rows whose ray passes through
// its voxel inside [a, b] and takes the piece length exactly as the forward
// projector cuts it.  FP64 sums, one write per voxel, no atomics.
//
// FUSED: instead of writing A^T z, finish the CG update of the voxel in the
// epilogue (q = A^T Lambda A p + p / sigma^2; x += alpha p; r -= alpha q) and
// write the workgroup's partial sum of r^2, so that q never goes to memory.
struct GatherUpdate {
    float *x, *r;
    const float *p;
    const double *scal;      // [SC_COUNT][nf]
    const double *consts;    // [0] = 1 / sigma^2
    double *part;            // [nf * tiles per frame]
};

// Length of the ray with crossing slope im (see zplane_s) inside z slab
// [klo, klo + 1] and xy piece [fa, fb] of a column whose source sits at
// s = -sf, up to its sign: the slab's two plane crossings e1, e2 clamped to
// the piece, subtracted.  Its magnitude is the length (0 when disjoint).  For
// zp = 0 the table holds a huge finite slope, so the slab holding z = 0 gets
// the whole piece and every other slab nothing, as in the forward walk.
//
// With e_lo = min(e1, e2) and e_hi = max(e1, e2) the length is
// max(min(fb, e_hi) - max(fa, e_lo), 0).  Clamping is monotone, so
// |clamp(e2, fa, fb) - clamp(e1, fa, fb)| = clamp(e_hi) - clamp(e_lo), and
// when the slab meets the piece clamp(e_hi) = min(fb, e_hi) and clamp(e_lo) =
// max(fa, e_lo): the same two FP32 values the forward projector subtracts, so
// the length is the same bit for bit; when they are disjoint both clamps are
// the same end of the piece and the difference is exactly 0.  The sign is
// dropped for free by the absolute-value source modifier of the multiply-add
// that uses the length.
__device__ __forceinline__ float slab_piece_signed(double im, double sf, double klo, float fa, float fb)
{
    const float e1 = (float)fma(klo, im, -sf), e2 = (float)fma(klo + 1.0, im, -sf);
    return __builtin_amdgcn_fmed3f(e2, fa, fb) - __builtin_amdgcn_fmed3f(e1, fa, fb);
}

// Detector columns [iu0, iu1] whose xy line can meet cell (ix, iy) in view v:
// the projections of the cell's four corners, widened by 1e-3 column.
__device__ __forceinline__ void cell_columns(const ProjParams &P, int64_t v, int ix, int iy, int &iu0, int &iu1)
{
    const float x0 = ix - 0.5f * P.nx, y0 = iy - 0.5f * P.ny;
    const float cu = 0.5f * (P.nu - 1);
    const float rs = (float)P.rs, rsd = (float)P.rsd;
    const float inv_du = (float)(1.0 / P.du), offu = (float)P.offu;
    const double2 cs = P.cs[v];
    const float c = (float)cs.x, s = (float)cs.y;
    float ulo = INFINITY, uhi = -INFINITY;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float X = x0 + (q & 1), Y = y0 + (q >> 1);
        const float b = Y * c - X * s;             // along e_u
        const float a = rs - (X * c + Y * s);      // depth from the source (> 0)
        const float fu = (rsd * b * __builtin_amdgcn_rcpf(a) - offu) * inv_du + cu;
        ulo = fminf(ulo, fu);
        uhi = fmaxf(uhi, fu);
    }
    iu0 = max((int)ceilf(ulo - 1e-3f), 0);
    iu1 = min((int)floorf(uhi + 1e-3f), P.nu - 1);
}

// Piece [fa, fb] of column E's xy line inside cell (ix, iy), with the forward
// walk's crossing expressions (so the lengths match A's bit for bit), and the
// detector rows per unit of z at the piece's two ends (the ray of height zp
// on the detector is at z = zp (s + sf) / lxy), smaller one in rmin, larger
// in rmax: rows through a voxel [z, z + 1] lie between z * rmin and
// (z + 1) * rmax for z >= 0, between z * rmax and (z + 1) * rmin below.
// False when the line misses the cell.
__device__ __forceinline__ bool cell_piece(const ColEntry &E, int ix, int iy, float inv_dv, float &fa, float &fb,
                                           float &rmin, float &rmax)
{
    if (!E.hit) return false;
    // a line parallel to an axis stays in one cell row
    const bool xok = E.iex != 0.0, yok = E.iey != 0.0;
    if ((!xok && ix != E.ixf) || (!yok && iy != E.iyf)) return false;
    const double px0 = plane_s(ix, E.iex, E.cx), px1 = plane_s(ix + 1, E.iex, E.cx);
    const double py0 = plane_s(iy, E.iey, E.cy), py1 = plane_s(iy + 1, E.iey, E.cy);
    const double xlo = xok ? fmin(px0, px1) : -INFINITY, xhi = xok ? fmax(px0, px1) : INFINITY;
    const double ylo = yok ? fmin(py0, py1) : -INFINITY, yhi = yok ? fmax(py0, py1) : INFINITY;
    const double sa = fmax(fmax(xlo, ylo), E.s_in), sb = fmin(fmin(xhi, yhi), E.s_out);
    fa = (float)sa;
    fb = (float)sb;
    if (!(fb > fa)) return false;
    const float lxyf = (float)E.lxy;
    const float ka = lxyf * __builtin_amdgcn_rcpf((float)(sa + E.sf));
    const float kb = lxyf * __builtin_amdgcn_rcpf((float)(sb + E.sf));
    rmin = fminf(ka, kb) * inv_dv;
    rmax = fmaxf(ka, kb) * inv_dv;
    return true;
}

// Per (view, xy cell) table of the pieces of the columns that meet the cell:
// hdr = their number n, ent[0..n-1] = their pieces in increasing column order.
// Built once per plan from the same cell_columns / cell_piece code the
// on-the-fly gather runs, so both adjoints see identical pieces.
__global__ void k_cell_table(const ProjParams P, int64_t n_views, int32_t *__restrict__ hdr,
                             CellEntry *__restrict__ ent, int K, int32_t *__restrict__ overflow)
{
    const int64_t ncell = (int64_t)P.nx * P.ny;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_views * ncell) return;
    const int64_t v = i / ncell;
    const int cell = (int)(i - v * ncell);
    const int ix = cell % P.nx, iy = cell / P.nx;
    int iu0, iu1;
    cell_columns(P, v, ix, iy, iu0, iu1);
    const float inv_dv = (float)(1.0 / P.dv);
    int n = 0;
    for (int iu = iu0; iu <= iu1; ++iu) {
        const ColEntry &E = P.cols[v * P.nu + iu];
        CellEntry c;
        if (!cell_piece(E, ix, iy, inv_dv, c.fa, c.fb, c.rmin, c.rmax)) continue;
        c.sf = E.sf;
        c.iu = iu;
        c.pad = 0;
        if (n < K) ent[i * K + n] = c;
        ++n;
    }
    for (int e = n; e < K; ++e) ent[i * K + e] = CellEntry{0.0f, 0.0f, 0.0f, 0.0f, 0.0, 0, 0};
    hdr[i] = min(n, K);
    if (n > K) atomicAdd(overflow, 1);
}

// The voxels of one lane (lower z face zlo[k], as a float and an exact double
// klo[k]) against column iu's piece [fa, fb]: add length * pre-scaled
// sinogram value of every detector row whose ray passes through the voxel
// inside the piece.  In two phases, so that a caller can issue the loads of
// several columns before their arithmetic: column_load finds every voxel's
// first candidate row and loads the first two candidates, column_sum takes
// the lengths (and reads any further rows).
template <int ZPL>
struct ColumnRows {
    __amdgpu_buffer_rsrc_t srow, irow;   // the column's sinogram values and crossing slopes
    int iva[ZPL];
    double ima[ZPL], imb[ZPL];
    float sva[ZPL], svb[ZPL];
};

// A lane's voxel faces: zlo = the lower face's height (a float, exact), and
// its split zpos = max(zlo, 0), zneg = min(zlo, 0) (one of them is 0).
template <int ZPL>
struct LaneZ {
    float zpos[ZPL], zneg[ZPL];
};

template <int ZPL>
__device__ __forceinline__ void column_load(const ProjParams &P, const float *sino_v, int iu, float rmin, float rmax,
                                            const float (&zlo)[ZPL], const LaneZ<ZPL> &L, float c_lo,
                                            ColumnRows<ZPL> &C)
{
    // sino_v: the view's sinogram; nu * nv < 2^31, so the column offset is 32-bit
    const int coff = iu * P.nv;
    C.srow = row_rsrc(sino_v + coff, P.nv * 4);
    C.irow = row_rsrc(P.imtab + coff, P.nv * 8);
#pragma unroll
    for (int k = 0; k < ZPL; ++k) {
        // the lowest row through [zlo, zlo + 1] within the piece: zlo * rmin above
        // z = 0, zlo * rmax below, as two multiply-adds of which one adds an exact
        // 0; at least the first row that can meet the volume (so the byte offsets
        // stay >= 0).  c_lo: the row coordinate at z = 0, widened by 1e-3 row.
        const float rc = fmaf(L.zneg[k], rmax, fmaf(L.zpos[k], rmin, c_lo));
        C.iva[k] = max((int)ceilf(rc), P.iv_lo);
    }
    // the first two candidate rows of every voxel without a branch.  Reads past a
    // row give 0, and a row outside [iva, ivb] misses the voxel inside the piece, so
    // its length is 0.  (Lanes past nz are never written back.)
#pragma unroll
    for (int k = 0; k < ZPL; ++k) {
        C.ima[k] = row_f64(C.irow, C.iva[k]);
        C.imb[k] = row_f64_next(C.irow, C.iva[k]);
        C.sva[k] = row_f32(C.srow, C.iva[k]);
        C.svb[k] = row_f32_next(C.srow, C.iva[k]);
    }
}

// MR = false: the plan's bound says no ray meets one voxel inside one piece in
// three or more rows, and the path for rows past the first two is not compiled;
// MR = true keeps it behind the plan's run-time flag.
template <int ZPL, bool MR>
__device__ __forceinline__ void column_sum(const ProjParams &P, const ColumnRows<ZPL> &C, double sf, float fa,
                                           float fb, float rmin, float rmax, const float (&zlo)[ZPL],
                                           const double (&klo)[ZPL], float (&vacc)[ZPL])
{
#pragma unroll
    for (int k = 0; k < ZPL; ++k) {
        const float la = slab_piece_signed(C.ima[k], sf, klo[k], fa, fb);
        const float lb = slab_piece_signed(C.imb[k], sf, klo[k], fa, fb);
        float acc_k = fmaf(fabsf(lb), C.svb[k], fmaf(fabsf(la), C.sva[k], vacc[k]));
        if (MR && P.multi_row) {
            // geometries where a ray can meet a voxel in three or more rows: the further candidates
            const float c_hi = (float)(0.5 * (P.nv - 1) - P.offv / P.dv) + 1e-3f;
            const float zhi = zlo[k] + 1.0f;
            const float r = zhi >= 0.0f ? rmax : rmin;
            const int ivb = min((int)floorf(fmaf(zhi, r, c_hi)), P.iv_hi);
            for (int ivr = C.iva[k] + 2; ivr <= ivb; ++ivr) {
                const float l = fabsf(slab_piece_signed(row_f64(C.irow, ivr), sf, klo[k], fa, fb));
                if (l > 0.0f) acc_k = fmaf(l, row_f32(C.srow, ivr), acc_k);
            }
        }
        vacc[k] = acc_k;
    }
}

template <int ZPL, bool MR>
__device__ __forceinline__ void gather_column(const ProjParams &P, const float *sino_v, int iu, double sf,
                                              float fa, float fb, float rmin, float rmax, const float (&zlo)[ZPL],
                                              const LaneZ<ZPL> &L, float c_lo, const double (&klo)[ZPL],
                                              float (&vacc)[ZPL])
{
    ColumnRows<ZPL> C;
    column_load<ZPL>(P, sino_v, iu, rmin, rmax, zlo, L, c_lo, C);
    column_sum<ZPL, MR>(P, C, sf, fa, fb, rmin, rmax, zlo, klo, vacc);
}

// KT = 0: the pieces are computed on the fly (back_mode 1); KT = 2, 3: they
// come from the cell table with KT slots per (view, cell) (back_mode 2), the
// next view's entries loaded while the current view is processed.
template <int ZPL, bool FUSED, int KT, bool MR>
__global__ __launch_bounds__(256) void k_back_gather(const ProjParams P, const float *__restrict__ sino,
                                                     double *__restrict__ out, const GatherUpdate U)
{
    const int nwaves = blockDim.x / WAVE;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x % WAVE;
    // the tile decode is wave-uniform: keep its results in scalar registers, so
    // the table and sinogram addresses derived from them stay scalar too.  The
    // launchers keep the grid below 2^31 workgroups, so the decode runs in 32
    // bits (64-bit divisions cost some 380 scalar instructions of code).
    const uint32_t t = (uint32_t)logical_tile(blockIdx.x, gridDim.x, P.xcd_remap);
    const uint32_t tpf = (uint32_t)P.g_tiles_per_frame;
    const int f = __builtin_amdgcn_readfirstlane((int)(t / tpf));
    uint32_t local = t - (uint32_t)f * tpf;
    const uint32_t nxg = (uint32_t)((P.nx + nwaves - 1) / nwaves);
    const int xg = __builtin_amdgcn_readfirstlane((int)(local % nxg));
    local /= nxg;
    const int iy = __builtin_amdgcn_readfirstlane((int)(local % (uint32_t)P.ny));
    const int zc = __builtin_amdgcn_readfirstlane((int)(local / (uint32_t)P.ny));
    const int ix = xg * nwaves + wave;
    if (P.active && !P.active[f]) return;   // the whole workgroup belongs to frame f
    const bool col_ok = ix < P.nx;
    int iz[ZPL];
    double klo[ZPL];
    float zlo[ZPL];
    LaneZ<ZPL> L;
    double acc[ZPL];
#pragma unroll
    for (int k = 0; k < ZPL; ++k) {
        iz[k] = (zc * ZPL + k) * WAVE + lane;
        klo[k] = (double)iz[k] - 0.5 * P.nz;
        zlo[k] = (float)klo[k];
        L.zpos[k] = fmaxf(zlo[k], 0.0f);
        L.zneg[k] = fminf(zlo[k], 0.0f);
        acc[k] = 0.0;
    }
    // FUSED: the CG update's p, x and r of the lane's voxels are loaded before
    // the views, so that their latency hides behind the gather instead of
    // ending every wave (128^3 x 16: 778 -> 744 us; 512 x 512 x 256: 55.1 ->
    // 53.6 ms, despite 4 waves per SIMD instead of 5 at 4 voxels per lane).
    // Only this lane writes these voxels, and only after the views.
    float pre_p[ZPL], pre_x[ZPL], pre_r[ZPL];
    if constexpr (FUSED) {
        const int64_t col0 = (int64_t)f * P.nvox + (int64_t)(iy * P.nx + (col_ok ? ix : 0)) * P.nz;
#pragma unroll
        for (int k = 0; k < ZPL; ++k) {
            const int64_t i0 = col0 + (col_ok && iz[k] < P.nz ? iz[k] : 0);
            pre_p[k] = U.p[i0];
            pre_x[k] = U.x[i0];
            pre_r[k] = U.r[i0];
        }
    }
    // detector row coordinate at z = 0 (row = z * rows-per-z + c), widened by 1e-3 row
    const float c_lo = (float)(0.5 * (P.nv - 1) - P.offv / P.dv) - 1e-3f;
    // views of the frame (fewer than 2^31 in all)
    const int v0 = __builtin_amdgcn_readfirstlane(col_ok ? (int)P.view_offset[f] : 0);
    const int v1 = __builtin_amdgcn_readfirstlane(col_ok ? (int)P.view_offset[f + 1] : 0);
    const int64_t view_len = (int64_t)P.nu * P.nv;
    if constexpr (KT > 0) {
        const int64_t ncell = (int64_t)P.nx * P.ny;
        const int64_t cell = (int64_t)iy * P.nx + ix;
        // the (view, cell) slots of consecutive views are ncell apart
        const int32_t *hdr = P.cell_hdr + v0 * ncell + cell;
        const CellEntry *ent = P.cell_ent + (v0 * ncell + cell) * KT;
        const float *sino_v = sino + v0 * view_len;
        if constexpr (ZPL <= 2) {
            // Views go in pairs (a, b).  The first slot of a view is processed
            // without a branch: when no column meets the cell it holds a zero
            // piece (fa = fb = 0), whose lengths are exactly 0, and so does the
            // missing b of an odd last pair (reading view a's sinogram).  Both
            // first slots' rows are loaded before either view's sums are taken.
            // Each view keeps its own FP32 sum, and they enter the FP64 sum in
            // view order, as one view at a time would.  The next pair's table
            // entries are loaded while the current pair is processed.
            const CellEntry zero{0.0f, 0.0f, 0.0f, 0.0f, 0.0, 0, 0};
            int na_next = 0, nb_next = 0;
            CellEntry ea_next = zero, eb_next = zero;
            if (v0 < v1) {
                na_next = hdr[0];
                ea_next = ent[0];
            }
            if (v0 + 1 < v1) {
                nb_next = hdr[ncell];
                eb_next = ent[ncell * KT];
            }
            for (int v = v0; v < v1; v += 2, sino_v += 2 * view_len) {
                const bool has_b = v + 1 < v1;
                const int na = na_next, nb = nb_next;
                const CellEntry ea = ea_next, eb = eb_next;
                const CellEntry *ent_a = ent, *ent_b = ent + ncell * KT;
                hdr += 2 * ncell;
                ent += 2 * ncell * KT;
                na_next = 0;
                nb_next = 0;
                ea_next = zero;
                eb_next = zero;
                if (v + 2 < v1) {
                    na_next = hdr[0];
                    ea_next = ent[0];
                }
                if (v + 3 < v1) {
                    nb_next = hdr[ncell];
                    eb_next = ent[ncell * KT];
                }
                const float *sino_b = has_b ? sino_v + view_len : sino_v;
                float va[ZPL], vb[ZPL];
#pragma unroll
                for (int k = 0; k < ZPL; ++k) {
                    va[k] = 0.0f;
                    vb[k] = 0.0f;
                }
                ColumnRows<ZPL> ca, cb;
                column_load<ZPL>(P, sino_v, ea.iu, ea.rmin, ea.rmax, zlo, L, c_lo, ca);
                column_load<ZPL>(P, sino_b, eb.iu, eb.rmin, eb.rmax, zlo, L, c_lo, cb);
                column_sum<ZPL, MR>(P, ca, ea.sf, ea.fa, ea.fb, ea.rmin, ea.rmax, zlo, klo, va);
                column_sum<ZPL, MR>(P, cb, eb.sf, eb.fa, eb.fb, eb.rmin, eb.rmax, zlo, klo, vb);
#pragma unroll
                for (int j = 1; j < KT; ++j) {
                    if (j >= na) break;
                    const CellEntry e = ent_a[j];
                    gather_column<ZPL, MR>(P, sino_v, e.iu, e.sf, e.fa, e.fb, e.rmin, e.rmax, zlo, L, c_lo, klo, va);
                }
#pragma unroll
                for (int j = 1; j < KT; ++j) {
                    if (j >= nb) break;
                    const CellEntry e = ent_b[j];
                    gather_column<ZPL, MR>(P, sino_b, e.iu, e.sf, e.fa, e.fb, e.rmin, e.rmax, zlo, L, c_lo, klo, vb);
                }
                // a missing b (odd last view) has a zero piece: vb is exactly +0
#pragma unroll
                for (int k = 0; k < ZPL; ++k) acc[k] += (double)va[k];
#pragma unroll
                for (int k = 0; k < ZPL; ++k) acc[k] += (double)vb[k];
            }
        } else {
            // Deeper columns (ZPL > 2) take one view at a time: two views' rows
            // in flight would cost more registers than the overlap gains.  The
            // next view's entries are loaded while the current one is processed.
            int n_next = 0;
            CellEntry e_next[KT];
            if (v0 < v1) {
                n_next = *hdr;
#pragma unroll
                for (int j = 0; j < KT; ++j) e_next[j] = ent[j];
            }
            for (int v = v0; v < v1; ++v, sino_v += view_len) {
                const int n = n_next;
                CellEntry ec[KT];
#pragma unroll
                for (int j = 0; j < KT; ++j) ec[j] = e_next[j];
                if (v + 1 < v1) {
                    hdr += ncell;
                    ent += ncell * KT;
                    n_next = *hdr;
#pragma unroll
                    for (int j = 0; j < KT; ++j) e_next[j] = ent[j];
                }
                float vacc[ZPL];
#pragma unroll
                for (int k = 0; k < ZPL; ++k) vacc[k] = 0.0f;
#pragma unroll
                for (int j = 0; j < KT; ++j) {
                    if (j >= n) break;
                    gather_column<ZPL, MR>(P, sino_v, ec[j].iu, ec[j].sf, ec[j].fa, ec[j].fb, ec[j].rmin, ec[j].rmax,
                                       zlo, L, c_lo, klo, vacc);
                }
#pragma unroll
                for (int k = 0; k < ZPL; ++k) acc[k] += (double)vacc[k];
            }
        }
    } else {
        const float inv_dv = (float)(1.0 / P.dv);
        for (int v = v0; v < v1; ++v) {
            float vacc[ZPL];
#pragma unroll
            for (int k = 0; k < ZPL; ++k) vacc[k] = 0.0f;
            int iu0, iu1;
            cell_columns(P, v, ix, iy, iu0, iu1);
            iu0 = __builtin_amdgcn_readfirstlane(iu0);
            iu1 = __builtin_amdgcn_readfirstlane(iu1);
            for (int iu = iu0; iu <= iu1; ++iu) {
                const ColEntry &E = P.cols[v * P.nu + iu];
                float fa, fb, rmin, rmax;
                if (!cell_piece(E, ix, iy, inv_dv, fa, fb, rmin, rmax)) continue;
                gather_column<ZPL, MR>(P, sino + v * view_len, iu, E.sf, fa, fb, rmin, rmax, zlo, L, c_lo, klo, vacc);
            }
#pragma unroll
            for (int k = 0; k < ZPL; ++k) acc[k] += (double)vacc[k];
        }
    }
    const int64_t col = (int64_t)f * P.nvox + (int64_t)(iy * P.nx + (col_ok ? ix : 0)) * P.nz;
    if (!FUSED) {
        if (!col_ok) return;
#pragma unroll
        for (int k = 0; k < ZPL; ++k)
            if (iz[k] < P.nz) out[col + iz[k]] = acc[k];
        return;
    }
    const double is2 = U.consts[0];
    const double alpha = U.scal[SC_ALPHA * P.nf + f];
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < ZPL; ++k) {
        if (col_ok && iz[k] < P.nz) {
            const int64_t i = col + iz[k];
            const double pv = pre_p[k];
            const double q = acc[k] + pv * is2;
            U.x[i] = (float)((double)pre_x[k] + alpha * pv);
            const float rf = (float)((double)pre_r[k] - alpha * q);
            U.r[i] = rf;
            part += (double)rf * (double)rf;
        }
    }
    __shared__ double red[4];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < nwaves; ++w) sum += red[w];
        U.part[t] = sum;
    }
}

// sino[i] *= scale[i mod (nu nv)]
__global__ void k_prescale(float *__restrict__ sino, const float *__restrict__ scale, int64_t per_view, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        sino[i] *= scale[i % per_view];
}

template <int R, bool STEEP, bool WT>
hipError_t fwd_dispatch_wt(const ProjParams &pp, int mode, dim3 grid, dim3 block, const float *vol,
                           const float *lam, const float *y, float *out, double *part, hipStream_t s)
{
    switch (mode) {
    case PM_PLAIN: hipLaunchKernelGGL((k_forward<R, PM_PLAIN, STEEP, WT>), grid, block, 0, s, pp, vol, lam, y, out, part); break;
    case PM_WEIGHTED: hipLaunchKernelGGL((k_forward<R, PM_WEIGHTED, STEEP, WT>), grid, block, 0, s, pp, vol, lam, y, out, part); break;
    case PM_COUNT: hipLaunchKernelGGL((k_forward<R, PM_COUNT, STEEP, WT>), grid, block, 0, s, pp, vol, lam, y, out, part); break;
    default: hipLaunchKernelGGL((k_forward<R, PM_RESID, STEEP, WT>), grid, block, 0, s, pp, vol, lam, y, out, part); break;
    }
    return hipGetLastError();
}

template <int R, bool STEEP>
hipError_t fwd_dispatch_mode(const ProjParams &pp, int mode, dim3 grid, dim3 block, const float *vol,
                             const float *lam, const float *y, float *out, double *part, hipStream_t s)
{
    if (pp.walk_head) return fwd_dispatch_wt<R, STEEP, true>(pp, mode, grid, block, vol, lam, y, out, part, s);
    return fwd_dispatch_wt<R, STEEP, false>(pp, mode, grid, block, vol, lam, y, out, part, s);
}

}  // namespace

ProjParams msf_plan::proj_params(bool with_active) const
{
    ProjParams pp{};
    pp.nx = nx; pp.ny = ny; pp.nz = nz; pp.nu = nu; pp.nv = nv; pp.nf = nf;
    pp.du = du; pp.dv = dv; pp.rs = rs; pp.rsd = rsd; pp.offu = offu; pp.offv = offv;
    pp.cs = d_cs;
    pp.view_offset = d_view_offset;
    pp.tile_offset = d_tile_offset;
    pp.active = with_active ? iscal + IS_ACTIVE * nf : nullptr;
    pp.n_ug = (nu + tiles.waves_per_group - 1) / tiles.waves_per_group;
    pp.rows_per_chunk = WAVE * tiles.rays_per_lane;
    pp.iv_lo = iv_lo;
    pp.iv_hi = iv_hi;
    pp.multi_row = multi_row ? 1 : 0;
    pp.n_vc = iv_hi >= iv_lo ? (iv_hi - iv_lo + pp.rows_per_chunk) / pp.rows_per_chunk : 0;
    pp.xcd_remap = tiles.xcd_remap;
    pp.nvox = nvox;
    pp.total_tiles = total_tiles();
    pp.rzp = d_rzp;
    pp.imtab = d_imtab;
    pp.cell_hdr = d_cell_hdr;
    pp.cell_ent = d_cell_ent;
    pp.cell_k = cell_k;
    pp.walk_head = tiles.back_mode == 2 ? d_walk_head : nullptr;
    pp.walk_ent = d_walk_ent;
    pp.walk_stride = nx + ny + 2;
    pp.cols = d_cols;
    pp.g_zpl = std::min(4, (nz + WAVE - 1) / WAVE);   // one wave per voxel column up to nz = 256
    pp.scale = d_scale;
    const int gw = tiles.waves_per_group;
    pp.g_tiles_per_frame = (int64_t)((nx + gw - 1) / gw) * ny * ((nz + WAVE * pp.g_zpl - 1) / (WAVE * pp.g_zpl));
    return pp;
}

hipError_t launch_forward(const msf_plan &P, int mode, const float *vol, const float *y, float *out,
                          bool with_active, hipStream_t s)
{
    const ProjParams pp = P.proj_params(with_active);
    if (pp.total_tiles == 0) return hipSuccess;
    const dim3 grid((unsigned)pp.total_tiles), block(WAVE * P.tiles.waves_per_group);
    if (P.steep) return fwd_dispatch_mode<1, true>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    switch (P.tiles.rays_per_lane) {
    case 1: return fwd_dispatch_mode<1, false>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    case 2: return fwd_dispatch_mode<2, false>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    case 3: return fwd_dispatch_mode<3, false>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    case 4: return fwd_dispatch_mode<4, false>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    case 5: return fwd_dispatch_mode<5, false>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    default: return fwd_dispatch_mode<6, false>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    }
}

hipError_t launch_back_scatter(const msf_plan &P, const float *sino, double *vol_acc, bool with_active,
                               hipStream_t s)
{
    const ProjParams pp = P.proj_params(with_active);
    if (pp.total_tiles == 0) return hipSuccess;
    const dim3 grid((unsigned)pp.total_tiles), block(WAVE * P.tiles.waves_per_group);
    if (P.steep) {
        hipLaunchKernelGGL((k_back_scatter<1, true>), grid, block, 0, s, pp, sino, vol_acc);
        return hipGetLastError();
    }
    switch (P.tiles.rays_per_lane) {
    case 1: hipLaunchKernelGGL((k_back_scatter<1, false>), grid, block, 0, s, pp, sino, vol_acc); break;
    case 2: hipLaunchKernelGGL((k_back_scatter<2, false>), grid, block, 0, s, pp, sino, vol_acc); break;
    case 3: hipLaunchKernelGGL((k_back_scatter<3, false>), grid, block, 0, s, pp, sino, vol_acc); break;
    case 4: hipLaunchKernelGGL((k_back_scatter<4, false>), grid, block, 0, s, pp, sino, vol_acc); break;
    case 5: hipLaunchKernelGGL((k_back_scatter<5, false>), grid, block, 0, s, pp, sino, vol_acc); break;
    default: hipLaunchKernelGGL((k_back_scatter<6, false>), grid, block, 0, s, pp, sino, vol_acc); break;
    }
    return hipGetLastError();
}

namespace {

template <bool FUSED, int KT>
void gather_dispatch(int zpl, dim3 grid, dim3 block, hipStream_t s, const ProjParams &pp, const float *sino,
                     double *out, const GatherUpdate &U)
{
    // Columns of up to 2 voxels per lane drop the third-row path when the plan's
    // bound allows (fewer registers, no hoisted row bound; 794 -> 776 us at
    // 128^3 x 16).  The deeper columns keep it behind the run-time flag: compiled
    // without it they run at 7 waves per SIMD instead of 5 and take 1-3% longer
    // (256^3 and 512 x 512 x 256), with the occupancy capped at 5 or 6 as well.
    const bool lean = !pp.multi_row;
    switch (zpl) {
    case 1:
        if (lean) hipLaunchKernelGGL((k_back_gather<1, FUSED, KT, false>), grid, block, 0, s, pp, sino, out, U);
        else hipLaunchKernelGGL((k_back_gather<1, FUSED, KT, true>), grid, block, 0, s, pp, sino, out, U);
        break;
    case 2:
        if (lean) hipLaunchKernelGGL((k_back_gather<2, FUSED, KT, false>), grid, block, 0, s, pp, sino, out, U);
        else hipLaunchKernelGGL((k_back_gather<2, FUSED, KT, true>), grid, block, 0, s, pp, sino, out, U);
        break;
    case 3: hipLaunchKernelGGL((k_back_gather<3, FUSED, KT, true>), grid, block, 0, s, pp, sino, out, U); break;
    default: hipLaunchKernelGGL((k_back_gather<4, FUSED, KT, true>), grid, block, 0, s, pp, sino, out, U); break;
    }
}

template <bool FUSED>
hipError_t gather_launch(const msf_plan &P, const ProjParams &pp, dim3 grid, dim3 block, hipStream_t s,
                         const float *sino, double *out, const GatherUpdate &U)
{
    if (P.tiles.back_mode == 2) {
        if (!pp.cell_hdr) return hipErrorInvalidValue;   // the cell table is built by setup_tiles
        if (pp.cell_k == 2) gather_dispatch<FUSED, 2>(pp.g_zpl, grid, block, s, pp, sino, out, U);
        else if (pp.cell_k == 3) gather_dispatch<FUSED, 3>(pp.g_zpl, grid, block, s, pp, sino, out, U);
        else return hipErrorInvalidValue;
    } else {
        gather_dispatch<FUSED, 0>(pp.g_zpl, grid, block, s, pp, sino, out, U);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_back_gather(const msf_plan &P, const float *sino, double *vol_out, bool with_active,
                              hipStream_t s)
{
    const ProjParams pp = P.proj_params(with_active);
    const int64_t total = pp.g_tiles_per_frame * P.nf;
    if (total == 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidValue;   // the kernel decodes tiles in 32 bits
    const dim3 grid((unsigned)total), block(WAVE * P.tiles.waves_per_group);
    const GatherUpdate U{};
    return gather_launch<false>(P, pp, grid, block, s, sino, vol_out, U);
}

hipError_t launch_back_gather_update(const msf_plan &P, hipStream_t s)
{
    const ProjParams pp = P.proj_params(true);
    const int64_t total = pp.g_tiles_per_frame * P.nf;
    if (total == 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidValue;   // the kernel decodes tiles in 32 bits
    if (total > P.part_g_per_frame * P.nf) return hipErrorInvalidValue;   // partial buffer sized for other tiles
    const dim3 grid((unsigned)total), block(WAVE * P.tiles.waves_per_group);
    GatherUpdate U;
    U.x = P.x;
    U.r = P.r;
    U.p = P.p;
    U.scal = P.scal;
    U.consts = P.consts;
    U.part = P.part_g;
    return gather_launch<true>(P, pp, grid, block, s, P.sz, nullptr, U);
}

hipError_t launch_walk_table(msf_plan &P, hipStream_t s)
{
    ProjParams pp = P.proj_params(false);
    const int64_t n = P.n_views * P.nu;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk_table, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, pp, n, P.d_walk_head,
                       P.d_walk_ent);
    return hipGetLastError();
}

hipError_t launch_cell_table(msf_plan &P, hipStream_t s)
{
    const ProjParams pp = P.proj_params(false);
    const int64_t n = P.n_views * (int64_t)P.nx * P.ny;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pp, P.n_views, P.d_cell_hdr,
                       P.d_cell_ent, P.cell_k, P.flags + 4);
    return hipGetLastError();
}

hipError_t launch_prescale(const msf_plan &P, float *sino, hipStream_t s)
{
    const int64_t n = P.nmeas_total;
    if (n == 0) return hipSuccess;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_prescale, dim3((unsigned)g), dim3(256), 0, s, sino, P.d_scale, (int64_t)P.nu * P.nv, n);
    return hipGetLastError();
}

hipError_t launch_back(const msf_plan &P, const float *sino, double *vol, bool with_active, hipStream_t s)
{
    if (P.tiles.back_mode != 0) return launch_back_gather(P, sino, vol, with_active, s);
    return launch_back_scatter(P, sino, vol, with_active, s);
}

hipError_t launch_col_table(msf_plan &P, hipStream_t s)
{
    const ProjParams pp = P.proj_params(false);
    const int64_t n = P.n_views * P.nu;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_col_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pp, P.n_views, P.d_cols);
    return hipGetLastError();
}
