// FP64 ray traversal of the refinement residual (exact.hip), callable from
// host and device code.  See exact.hip for what it computes.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

struct ExactArgs {
    int nx, ny, nz, nu, nv, nf;
    double du, dv, rs, rsd, offu, offv;
    const double2 *cs;           // [n_views] (cos t, sin t)
    const int64_t *view_offset;  // [nf + 1]
    int64_t n_views, nvox;
};

// Source and direction of ray (view, iu, iv): S + t d reaches the pixel centre at t = 1.
__host__ __device__ inline void ray_of(const ExactArgs &A, int64_t view, int iu, int iv, double S[3], double d[3])
{
    const double2 cs = A.cs[view];
    const double u = (iu - 0.5 * (A.nu - 1)) * A.du + A.offu;
    const double v = (iv - 0.5 * (A.nv - 1)) * A.dv + A.offv;
    S[0] = A.rs * cs.x;
    S[1] = A.rs * cs.y;
    S[2] = 0.0;
    d[0] = -A.rsd * cs.x - u * cs.y;
    d[1] = -A.rsd * cs.y + u * cs.x;
    d[2] = v;
}

// Calls op(voxel index within the frame, FP64 length) for every piece of the ray inside the volume.
template <class Op>
__host__ __device__ inline void traverse(const ExactArgs &A, const double S[3], const double d[3], Op &&op)
{
    const int n[3] = {A.nx, A.ny, A.nz};
    const double h[3] = {0.5 * A.nx, 0.5 * A.ny, 0.5 * A.nz};
    double inv[3], tnext[3];
    int m[3], step[3];
    double t_in = 0.0, t_out = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            inv[a] = 1.0 / d[a];
            double t0 = (-h[a] - S[a]) * inv[a], t1 = (h[a] - S[a]) * inv[a];
            if (t0 > t1) {
                const double t = t0;
                t0 = t1;
                t1 = t;
            }
            t_in = fmax(t_in, t0);
            t_out = fmin(t_out, t1);
        } else {
            inv[a] = 0.0;
            if (!(S[a] >= -h[a] && S[a] < h[a])) return;   // parallel to the slab and outside it
        }
    }
    if (!(t_out > t_in)) return;
    // first plane of each family beyond t_in, in the direction of travel
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            step[a] = 0;
            m[a] = 0;
            tnext[a] = INFINITY;
            continue;
        }
        step[a] = d[a] > 0.0 ? 1 : -1;
        const double c = S[a] + t_in * d[a] + h[a];   // plane coordinate at entry, in [0, n]
        int k = step[a] > 0 ? (int)floor(c) + 1 : (int)ceil(c) - 1;
        k = k < 0 ? 0 : (k > n[a] ? n[a] : k);
        double t = ((double)k - h[a] - S[a]) * inv[a];
        // rounding at the entry face: move on to the first plane strictly beyond t_in
        while (t <= t_in && k + step[a] >= 0 && k + step[a] <= n[a]) {
            k += step[a];
            t = ((double)k - h[a] - S[a]) * inv[a];
        }
        m[a] = k;
        tnext[a] = t > t_in ? t : INFINITY;
    }
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double t0 = t_in;
    for (int guard = n[0] + n[1] + n[2] + 3; guard > 0 && t0 < t_out; --guard) {
        const double t1 = fmin(fmin(fmin(tnext[0], tnext[1]), tnext[2]), t_out);
        if (t1 > t0) {
            const double tm = 0.5 * (t0 + t1);
            const int ix = (int)floor(S[0] + tm * d[0] + h[0]);
            const int iy = (int)floor(S[1] + tm * d[1] + h[1]);
            const int iz = (int)floor(S[2] + tm * d[2] + h[2]);
            if ((unsigned)ix < (unsigned)A.nx && (unsigned)iy < (unsigned)A.ny && (unsigned)iz < (unsigned)A.nz)
                op(((int64_t)iy * A.nx + ix) * A.nz + iz, (t1 - t0) * L);
        }
        for (int a = 0; a < 3; ++a) {
            if (tnext[a] <= t1) {
                m[a] += step[a];
                tnext[a] = (m[a] >= 0 && m[a] <= n[a]) ? ((double)m[a] - h[a] - S[a]) * inv[a] : INFINITY;
            }
        }
        t0 = t1;
    }
}

