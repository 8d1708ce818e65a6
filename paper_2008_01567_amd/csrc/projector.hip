// Cone-beam forward projector A and its adjoint A^T for gfx950.
//
// A[i][j] is the length of ray i (point source -> detector pixel centre)
// inside voxel j (paper Sec. II: the system matrix of eq. (LL_time_expand);
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
// The adjoint (scatter) runs the very same traversal and adds
// length * value into each voxel with hardware FP64 atomics (an FP64
// accumulator keeps the mixed-sign sums of CG free of FP32 cancellation), so
// A and A^T use bit-identical lengths: the adjoint is exact up to summation
// order.
#include "msf_internal.h"

#include <cmath>

namespace {

constexpr int WAVE = 64;

struct Column {
    double fx, fy;      // foot point of the xy line (closest approach to the z axis)
    double ex, ey;      // unit xy direction, source -> pixel
    double iex, iey;    // 1/ex, 1/ey (unused when the component is 0)
    double sf;          // xy distance source -> foot point (the source sits at s = -sf)
    double inv_lxy;     // 1 / (xy distance source -> pixel)
    double s_in, s_out; // xy-box clip of the line
    int ix, iy;         // entry cell
    int stepx, stepy;
    double sxn, syn;    // next x / y plane crossing
};

__device__ __forceinline__ bool column_setup(const ProjParams &P, int view, int iu, Column &c)
{
    const double2 cs = P.cs[view];
    const double u = (iu - 0.5 * (P.nu - 1)) * P.du + P.offu;
    const double sx = P.rs * cs.x, sy = P.rs * cs.y;
    const double dx = -P.rsd * cs.x - u * cs.y;
    const double dy = -P.rsd * cs.y + u * cs.x;
    const double lxy = sqrt(dx * dx + dy * dy);
    c.ex = dx / lxy;
    c.ey = dy / lxy;
    c.inv_lxy = 1.0 / lxy;
    c.sf = -(sx * c.ex + sy * c.ey);
    c.fx = sx + c.sf * c.ex;
    c.fy = sy + c.sf * c.ey;
    const double hx = 0.5 * P.nx, hy = 0.5 * P.ny;
    double sx0, sx1, sy0, sy1;
    if (c.ex != 0.0) {
        c.iex = 1.0 / c.ex;
        const double a = (-hx - c.fx) * c.iex, b = (hx - c.fx) * c.iex;
        sx0 = fmin(a, b);
        sx1 = fmax(a, b);
    } else {
        c.iex = 0.0;
        if (!(c.fx >= -hx && c.fx < hx)) return false;
        sx0 = -INFINITY;
        sx1 = INFINITY;
    }
    if (c.ey != 0.0) {
        c.iey = 1.0 / c.ey;
        const double a = (-hy - c.fy) * c.iey, b = (hy - c.fy) * c.iey;
        sy0 = fmin(a, b);
        sy1 = fmax(a, b);
    } else {
        c.iey = 0.0;
        if (!(c.fy >= -hy && c.fy < hy)) return false;
        sy0 = -INFINITY;
        sy1 = INFINITY;
    }
    c.s_in = fmax(sx0, sy0);
    c.s_out = fmin(sx1, sy1);
    if (!(c.s_out > c.s_in)) return false;
    c.stepx = c.ex > 0.0 ? 1 : (c.ex < 0.0 ? -1 : 0);
    c.stepy = c.ey > 0.0 ? 1 : (c.ey < 0.0 ? -1 : 0);
    // entry cell: the entering axis from the direction, the other from the entry point
    if (sx0 >= sy0) c.ix = c.stepx > 0 ? 0 : P.nx - 1;
    else c.ix = min(max((int)floor(c.fx + c.ex * c.s_in + hx), 0), P.nx - 1);
    if (sy0 >= sx0) c.iy = c.stepy > 0 ? 0 : P.ny - 1;
    else c.iy = min(max((int)floor(c.fy + c.ey * c.s_in + hy), 0), P.ny - 1);
    c.sxn = c.stepx > 0 ? ((c.ix + 1) - hx - c.fx) * c.iex
          : (c.stepx < 0 ? (c.ix - hx - c.fx) * c.iex : INFINITY);
    c.syn = c.stepy > 0 ? ((c.iy + 1) - hy - c.fy) * c.iey
          : (c.stepy < 0 ? (c.iy - hy - c.fy) * c.iey : INFINITY);
    return true;
}

// z-state of one ray (one detector row) along the shared xy line.
struct RayZ {
    double z0, im;      // z at the foot point; 1/m with m = dz/ds (0 if m == 0)
    float lzi, lzo;     // s-range inside the z slab of the volume
    float szn;          // next z-plane crossing
    float scale;        // 3D length per unit s: sqrt(1 + m^2)
    int iz, zstep;
};

__device__ __forceinline__ void ray_setup(const ProjParams &P, const Column &c, int iv, bool valid, RayZ &z)
{
    const double hz = 0.5 * P.nz;
    const double zp = (iv - 0.5 * (P.nv - 1)) * P.dv + P.offv;
    const double m = zp * c.inv_lxy;
    z.z0 = m * c.sf;
    z.scale = (float)sqrt(1.0 + m * m);
    double lzi, lzo;
    if (m != 0.0) {
        z.im = 1.0 / m;
        const double a = (-hz - z.z0) * z.im, b = (hz - z.z0) * z.im;
        lzi = fmin(a, b);
        lzo = fmax(a, b);
    } else {
        z.im = 0.0;
        const bool in = z.z0 >= -hz && z.z0 < hz;
        lzi = in ? -INFINITY : INFINITY;
        lzo = in ? INFINITY : -INFINITY;
    }
    z.zstep = m > 0.0 ? 1 : (m < 0.0 ? -1 : 0);
    const double start = fmax(c.s_in, lzi);
    if (!valid || !(fmin(c.s_out, lzo) > start)) {
        z.lzi = INFINITY;
        z.lzo = -INFINITY;
        z.iz = 0;
        z.szn = INFINITY;
        return;
    }
    z.lzi = (float)lzi;
    z.lzo = (float)lzo;
    if (lzi >= c.s_in) z.iz = z.zstep > 0 ? 0 : P.nz - 1;
    else z.iz = min(max((int)floor(z.z0 + m * c.s_in + hz), 0), P.nz - 1);
    z.szn = z.zstep > 0 ? (float)(((z.iz + 1) - hz - z.z0) * z.im)
          : (z.zstep < 0 ? (float)((z.iz - hz - z.z0) * z.im) : INFINITY);
}

// Walk the pieces of one ray inside the xy cell [a, b] of the current voxel
// column, calling op(iz, length) for each z voxel with a positive length.
template <class Op>
__device__ __forceinline__ void ray_cell(RayZ &z, float scur, float snext, int nz, double hz, Op &&op)
{
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
        z.szn = (float)(((z.zstep > 0 ? z.iz + 1 : z.iz) - hz - z.z0) * z.im);
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

template <int R, int MODE>
__global__ __launch_bounds__(256) void k_forward(const ProjParams P, const float *__restrict__ vol,
                                                 const float *__restrict__ lam, const float *__restrict__ y,
                                                 float *__restrict__ out, double *__restrict__ partial)
{
    const int nwaves = blockDim.x / WAVE;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t t = logical_tile(blockIdx.x, gridDim.x, P.xcd_remap);
    const Tile T = decode_tile(P, t, wave, nwaves);
    double part = 0.0;
    if (T.ok) {
        const double hz = 0.5 * P.nz;
        const float hxf = 0.5f * P.nx, hyf = 0.5f * P.ny;
        (void)hxf; (void)hyf;
        int iv[R];
        double acc[R];   // FP64 ray sums: the FP32 x FP32 products are exact in FP64
        RayZ z[R];
        Column c;
        const bool hit = column_setup(P, T.view, T.iu, c);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            iv[r] = P.iv_lo + T.vc * P.rows_per_chunk + r * WAVE + lane;
            acc[r] = 0.0;
            if (hit) ray_setup(P, c, iv[r], iv[r] <= P.iv_hi, z[r]);
        }
        if (hit) {
            const float *volf = vol + (int64_t)T.frame * P.nvox;
            const double hx = 0.5 * P.nx, hy = 0.5 * P.ny;
            double s_cur = c.s_in;
            float scur = (float)s_cur;
            int ix = c.ix, iy = c.iy;
            double sxn = c.sxn, syn = c.syn;
            for (int guard = P.nx + P.ny + 2; guard > 0; --guard) {
                const double s_next = fmin(fmin(sxn, syn), c.s_out);
                const float snext = (float)s_next;
                const float *colp = volf + (int64_t)(iy * P.nx + ix) * P.nz;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double a = acc[r];
                    if (MODE == PM_COUNT)
                        ray_cell(z[r], scur, snext, P.nz, hz, [&](int, float l) { a += l > 0.0f ? 1.0 : 0.0; });
                    else
                        ray_cell(z[r], scur, snext, P.nz, hz,
                                 [&](int iz, float l) { a = fma((double)l, (double)colp[iz], a); });
                    acc[r] = a;
                }
                if (s_next >= c.s_out) break;
                if (sxn <= syn) {
                    ix += c.stepx;
                    if ((unsigned)ix >= (unsigned)P.nx) break;
                    sxn = ((c.stepx > 0 ? ix + 1 : ix) - hx - c.fx) * c.iex;
                } else {
                    iy += c.stepy;
                    if ((unsigned)iy >= (unsigned)P.ny) break;
                    syn = ((c.stepy > 0 ? iy + 1 : iy) - hy - c.fy) * c.iey;
                }
                scur = snext;
            }
        }
        const int64_t base = (int64_t)T.view * P.nu * P.nv + (int64_t)T.iu * P.nv;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (iv[r] > P.iv_hi) continue;
            const int64_t idx = base + iv[r];
            const double w = hit ? acc[r] * (MODE == PM_COUNT ? 1.0 : (double)z[r].scale) : 0.0;
            if (MODE == PM_PLAIN || MODE == PM_COUNT) {
                out[idx] = (float)w;
            } else if (MODE == PM_WEIGHTED) {
                const double l = lam[idx];
                out[idx] = (float)(l * w);
                part += w * l * w;
            } else {
                out[idx] = (float)((double)lam[idx] * ((double)y[idx] - w));
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

template <int R>
__global__ __launch_bounds__(256) void k_back_scatter(const ProjParams P, const float *__restrict__ sino,
                                                      double *__restrict__ vol)
{
    const int nwaves = blockDim.x / WAVE;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t t = logical_tile(blockIdx.x, gridDim.x, P.xcd_remap);
    const Tile T = decode_tile(P, t, wave, nwaves);
    if (!T.ok) return;
    Column c;
    if (!column_setup(P, T.view, T.iu, c)) return;
    const double hz = 0.5 * P.nz;
    RayZ z[R];
    float val[R];
    const int64_t base = (int64_t)T.view * P.nu * P.nv + (int64_t)T.iu * P.nv;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iv = P.iv_lo + T.vc * P.rows_per_chunk + r * WAVE + lane;
        const bool valid = iv <= P.iv_hi;
        ray_setup(P, c, iv, valid, z[r]);
        val[r] = valid ? sino[base + iv] * z[r].scale : 0.0f;
        if (val[r] == 0.0f) {   // nothing to add: skip this ray's atomics
            z[r].lzi = INFINITY;
            z[r].lzo = -INFINITY;
        }
    }
    double *volf = vol + (int64_t)T.frame * P.nvox;
    const double hx = 0.5 * P.nx, hy = 0.5 * P.ny;
    float scur = (float)c.s_in;
    int ix = c.ix, iy = c.iy;
    double sxn = c.sxn, syn = c.syn;
    for (int guard = P.nx + P.ny + 2; guard > 0; --guard) {
        const double s_next = fmin(fmin(sxn, syn), c.s_out);
        const float snext = (float)s_next;
        double *colp = volf + (int64_t)(iy * P.nx + ix) * P.nz;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double v = val[r];
            ray_cell(z[r], scur, snext, P.nz, hz, [&](int iz, float l) { unsafeAtomicAdd(colp + iz, (double)l * v); });
        }
        if (s_next >= c.s_out) break;
        if (sxn <= syn) {
            ix += c.stepx;
            if ((unsigned)ix >= (unsigned)P.nx) break;
            sxn = ((c.stepx > 0 ? ix + 1 : ix) - hx - c.fx) * c.iex;
        } else {
            iy += c.stepy;
            if ((unsigned)iy >= (unsigned)P.ny) break;
            syn = ((c.stepy > 0 ? iy + 1 : iy) - hy - c.fy) * c.iey;
        }
        scur = snext;
    }
}

template <int R>
hipError_t fwd_dispatch_mode(const ProjParams &pp, int mode, dim3 grid, dim3 block, const float *vol,
                             const float *lam, const float *y, float *out, double *part, hipStream_t s)
{
    switch (mode) {
    case PM_PLAIN: hipLaunchKernelGGL((k_forward<R, PM_PLAIN>), grid, block, 0, s, pp, vol, lam, y, out, part); break;
    case PM_WEIGHTED: hipLaunchKernelGGL((k_forward<R, PM_WEIGHTED>), grid, block, 0, s, pp, vol, lam, y, out, part); break;
    case PM_COUNT: hipLaunchKernelGGL((k_forward<R, PM_COUNT>), grid, block, 0, s, pp, vol, lam, y, out, part); break;
    default: hipLaunchKernelGGL((k_forward<R, PM_RESID>), grid, block, 0, s, pp, vol, lam, y, out, part); break;
    }
    return hipGetLastError();
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
    pp.n_vc = iv_hi >= iv_lo ? (iv_hi - iv_lo + pp.rows_per_chunk) / pp.rows_per_chunk : 0;
    pp.xcd_remap = tiles.xcd_remap;
    pp.nvox = nvox;
    pp.total_tiles = total_tiles();
    return pp;
}

hipError_t launch_forward(const msf_plan &P, int mode, const float *vol, const float *y, float *out,
                          bool with_active, hipStream_t s)
{
    const ProjParams pp = P.proj_params(with_active);
    if (pp.total_tiles == 0) return hipSuccess;
    const dim3 grid((unsigned)pp.total_tiles), block(WAVE * P.tiles.waves_per_group);
    switch (P.tiles.rays_per_lane) {
    case 1: return fwd_dispatch_mode<1>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    case 2: return fwd_dispatch_mode<2>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    default: return fwd_dispatch_mode<4>(pp, mode, grid, block, vol, P.slam, y, out, P.part_proj, s);
    }
}

hipError_t launch_back_scatter(const msf_plan &P, const float *sino, double *vol_acc, bool with_active,
                               hipStream_t s)
{
    const ProjParams pp = P.proj_params(with_active);
    if (pp.total_tiles == 0) return hipSuccess;
    const dim3 grid((unsigned)pp.total_tiles), block(WAVE * P.tiles.waves_per_group);
    switch (P.tiles.rays_per_lane) {
    case 1: hipLaunchKernelGGL((k_back_scatter<1>), grid, block, 0, s, pp, sino, vol_acc); break;
    case 2: hipLaunchKernelGGL((k_back_scatter<2>), grid, block, 0, s, pp, sino, vol_acc); break;
    default: hipLaunchKernelGGL((k_back_scatter<4>), grid, block, 0, s, pp, sino, vol_acc); break;
    }
    return hipGetLastError();
}
