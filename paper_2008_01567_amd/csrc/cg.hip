// Batched conjugate gradients for the proximal map of the data term
// (paper Sec. III, eq. (4)), one independent system per time frame
// (the data term separates over frames, eq. (2)):
//     H_n = A_n^T Lambda_n A_n + sigma^-2 I,   b_n = A_n^T Lambda_n y_n + sigma^-2 v_n.
// Vectors are FP32 in HBM; every inner product, step size and residual norm
// is FP64.  Vector updates are evaluated in FP64 and rounded once to FP32.
//
// One CG step for all frames is six launches (five with the voxel-driven adjoint):
//   forward   w = A p, z = Lambda w, partial <w, Lambda w>   (projector.hip)
//   alpha     <p, H p> = <w, Lambda w> + ||p||^2 / sigma^2, alpha = gamma / <p, H p>
//   back      q' = A^T z (scatter into a zeroed buffer)
//   update    x += alpha p, r -= alpha (q' + p / sigma^2), q' = 0, partial ||r||^2
//             (with the voxel-driven adjoint, back and update are one kernel and q' stays in registers)
//   beta      gamma' = ||r||^2, convergence test, beta = gamma' / gamma
//   direction p = r + beta p, partial ||p||^2
// Per-frame FP64 partial sums are written per workgroup and reduced in a
// fixed order by one workgroup per frame (deterministic).  A frame whose
// relative residual reaches the tolerance (or max_iter) is switched off in
// a device-side mask; every kernel skips it, so its iterate stays frozen.
#include "msf_internal.h"

namespace {

constexpr int VB = 256;     // threads per volume-kernel block
constexpr int VE = 8;       // elements per thread
constexpr int VCHUNK = VB * VE;

__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[VB / 64];
    __syncthreads();   // the previous call's readers are done with red[]
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / 64); ++i) s += red[i];
    return s;   // valid on thread 0
}

// ------------------------------------------------------------ transpose --
__global__ void k_transpose(const float *__restrict__ in, float *__restrict__ out, int R, int C, int check,
                            int32_t *__restrict__ flags)
{
    __shared__ float tile[32][33];
    const int64_t b = blockIdx.z;
    const float *src = in + b * (int64_t)R * C;
    float *dst = out + b * (int64_t)R * C;
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    int bad = 0;
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int rr = r0 + k, cc = c0 + threadIdx.x;
        if (rr < R && cc < C) {
            const float v = src[(int64_t)rr * C + cc];
            tile[k][threadIdx.x] = v;
            if (check == 1) bad += !isfinite(v);
            else if (check == 2) bad += !(isfinite(v) && v >= 0.0f);
        }
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int cc = c0 + k, rr = r0 + threadIdx.x;
        if (rr < R && cc < C) dst[(int64_t)cc * R + rr] = tile[threadIdx.x][k];
    }
    if (check && bad) atomicAdd(flags, bad);
}

__global__ void k_fill(float *p, int64_t n, float v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_d(double *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_d2f(const double *__restrict__ s, float *__restrict__ d, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (float)s[i];
}

__global__ void k_copy(float *__restrict__ d, const float *__restrict__ s, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

// o = a * b * scale[i mod per_view]  (Lambda y pre-multiplied by the ray length factor for the adjoint)
__global__ void k_mul_scaled(const float *__restrict__ a, const float *__restrict__ b, const float *__restrict__ sc,
                             int64_t per_view, float *__restrict__ o, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        o[i] = (float)((double)a[i] * (double)b[i] * (double)sc[i % per_view]);
}

__global__ void k_mul(const float *__restrict__ a, const float *__restrict__ b, float *__restrict__ o, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        o[i] = a[i] * b[i];
}

unsigned grid_for(int64_t n)
{
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// ---------------------------------------------------------- volume ops --
struct VolArgs {
    float *x, *r, *p;
    double *bp;
    double *x64;             // FP64 iterate of a refined solve (or null)
    const float *vin;
    double *part;            // [nf * bpf]
    const double *scal;      // [SC_COUNT][nf]
    const int32_t *active;   // [nf] or nullptr
    const double *consts;
    int64_t nvox;
    int nf, bpf;
};

// ||b||^2 partials with b = A^T(Lambda y) (in bp) + v / sigma^2; clears bp.
__global__ __launch_bounds__(VB) void k_vol_bnorm(VolArgs A)
{
    const int f = blockIdx.y;
    const double is2 = A.consts[0];
    const int64_t base = (int64_t)f * A.nvox;
    double s = 0.0;
    for (int k = 0; k < VE; ++k) {
        const int64_t i = (int64_t)blockIdx.x * VCHUNK + k * VB + threadIdx.x;
        if (i < A.nvox) {
            const double b = A.bp[base + i] + (double)A.vin[base + i] * is2;
            s += b * b;
            A.bp[base + i] = 0.0;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) A.part[(int64_t)f * A.bpf + blockIdx.x] = s;
}

// r = A^T Lambda (y - A x) (in bp) + (v - x) / sigma^2 = b - H x;  clears bp.
// store 1: r = p = that residual; store 2: p only; store 0: only ||.||^2 partials.
__global__ __launch_bounds__(VB) void k_vol_residual(VolArgs A, int store)
{
    const int f = blockIdx.y;
    const double is2 = A.consts[0];
    const int64_t base = (int64_t)f * A.nvox;
    double s = 0.0;
    for (int k = 0; k < VE; ++k) {
        const int64_t i = (int64_t)blockIdx.x * VCHUNK + k * VB + threadIdx.x;
        if (i < A.nvox) {
            const double rv = A.bp[base + i] + ((double)A.vin[base + i] - (double)A.x[base + i]) * is2;
            const float rf = (float)rv;
            if (store == 1) A.r[base + i] = rf;
            if (store) A.p[base + i] = rf;
            s += store ? (double)rf * (double)rf : rv * rv;
            A.bp[base + i] = 0.0;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) A.part[(int64_t)f * A.bpf + blockIdx.x] = s;
}

// sum of bp per frame (partials), clears bp
__global__ __launch_bounds__(VB) void k_vol_sum_bp(VolArgs A)
{
    const int f = blockIdx.y;
    const int64_t base = (int64_t)f * A.nvox;
    double s = 0.0;
    for (int k = 0; k < VE; ++k) {
        const int64_t i = (int64_t)blockIdx.x * VCHUNK + k * VB + threadIdx.x;
        if (i < A.nvox) {
            s += A.bp[base + i];
            A.bp[base + i] = 0.0;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) A.part[(int64_t)f * A.bpf + blockIdx.x] = s;
}

// p = r / diag_f
__global__ __launch_bounds__(VB) void k_scale_feature(VolArgs A)
{
    const int f = blockIdx.y;
    const double inv = 1.0 / A.scal[SC_DIAG * A.nf + f];
    const int64_t base = (int64_t)f * A.nvox;
    for (int k = 0; k < VE; ++k) {
        const int64_t i = (int64_t)blockIdx.x * VCHUNK + k * VB + threadIdx.x;
        if (i < A.nvox) A.p[base + i] = (float)((double)A.r[base + i] * inv);
    }
}

// per frame: learned start kept (IS_CNN = 1): r = p; else x = v, p = r.
// Either way the ||p||^2 partials of the direction that is kept are
// rewritten, in the order k_vol_residual sums them, so the first step's
// <p, H p> uses that direction (a rejected frame continues bit for bit as
// the solve from v would).
__global__ __launch_bounds__(VB) void k_vol_select(VolArgs A, const int32_t *use_cnn)
{
    const int f = blockIdx.y;
    const bool keep = use_cnn[f] != 0;
    const int64_t base = (int64_t)f * A.nvox;
    double s = 0.0;
    for (int k = 0; k < VE; ++k) {
        const int64_t i = (int64_t)blockIdx.x * VCHUNK + k * VB + threadIdx.x;
        if (i < A.nvox) {
            float pf;
            if (keep) {
                pf = A.p[base + i];
                A.r[base + i] = pf;
            } else {
                pf = A.r[base + i];
                A.x[base + i] = A.vin[base + i];
                A.p[base + i] = pf;
            }
            s += (double)pf * (double)pf;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) A.part[(int64_t)f * A.bpf + blockIdx.x] = s;
}

// Iterative refinement: fold the FP32 correction into the FP64 iterate.
__global__ __launch_bounds__(VB) void k_fold(VolArgs A)
{
    const int f = blockIdx.y;
    const int64_t base = (int64_t)f * A.nvox;
    for (int k = 0; k < VE; ++k) {
        const int64_t i = (int64_t)blockIdx.x * VCHUNK + k * VB + threadIdx.x;
        if (i < A.nvox) {
            A.x64[base + i] += (double)A.x[base + i];
            A.x[base + i] = 0.0f;
        }
    }
}

// Iterative refinement: r = p = bp + (v - x64) / sigma^2 (bp the FP64
// A^T Lambda (y - A x64)), the residual of the FP64 iterate, rounded once to
// FP32; partial ||r||^2 of the rounded values; clears bp.
__global__ __launch_bounds__(VB) void k_vol_residual64(VolArgs A)
{
    const int f = blockIdx.y;
    const double is2 = A.consts[0];
    const int64_t base = (int64_t)f * A.nvox;
    double s = 0.0;
    for (int k = 0; k < VE; ++k) {
        const int64_t i = (int64_t)blockIdx.x * VCHUNK + k * VB + threadIdx.x;
        if (i < A.nvox) {
            const double rv = A.bp[base + i] + ((double)A.vin[base + i] - A.x64[base + i]) * is2;
            const float rf = (float)rv;
            A.r[base + i] = rf;
            A.p[base + i] = rf;
            s += (double)rf * (double)rf;
            A.bp[base + i] = 0.0;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) A.part[(int64_t)f * A.bpf + blockIdx.x] = s;
}

// x += alpha p;  r -= alpha (bp + p / sigma^2);  bp = 0;  partial ||r||^2.
__global__ __launch_bounds__(VB) void k_update_xr(VolArgs A)
{
    const int f = blockIdx.y;
    if (A.active && !A.active[f]) return;
    const double is2 = A.consts[0];
    const double alpha = A.scal[SC_ALPHA * A.nf + f];
    const int64_t base = (int64_t)f * A.nvox + (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
    const int64_t n = A.nvox - (int64_t)blockIdx.x * VCHUNK - threadIdx.x;   // elements k with k * VB < n
    // all of the thread's loads first: the stores below could alias them, so the
    // compiler would otherwise wait for each element's loads after the last store.
    // Elements past the frame's end read its first voxel (base itself can be past
    // the end of the last frame) and are not used.
    float pl[VE], xl[VE], rl[VE];
    double bl[VE];
#pragma unroll
    for (int k = 0; k < VE; ++k) {
        const bool in = (int64_t)k * VB < n;
        const int64_t i = in ? base + k * VB : (int64_t)f * A.nvox;
        pl[k] = A.p[i];
        xl[k] = A.x[i];
        rl[k] = A.r[i];
        bl[k] = A.bp[i];
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < VE; ++k) {
        if ((int64_t)k * VB < n) {
            const int64_t i = base + k * VB;
            const double pv = pl[k];
            const double q = bl[k] + pv * is2;
            A.x[i] = (float)((double)xl[k] + alpha * pv);
            const float rf = (float)((double)rl[k] - alpha * q);
            A.r[i] = rf;
            A.bp[i] = 0.0;
            s += (double)rf * (double)rf;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) A.part[(int64_t)f * A.bpf + blockIdx.x] = s;
}

// p = r + beta p;  partial ||p||^2.
__global__ __launch_bounds__(VB) void k_update_p(VolArgs A)
{
    const int f = blockIdx.y;
    if (A.active && !A.active[f]) return;
    const double beta = A.scal[SC_BETA * A.nf + f];
    const int64_t base = (int64_t)f * A.nvox + (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
    const int64_t n = A.nvox - (int64_t)blockIdx.x * VCHUNK - threadIdx.x;   // elements k with k * VB < n
    // all loads first, elements past the frame's end reading its first voxel (see k_update_xr)
    float rl[VE], pl[VE];
#pragma unroll
    for (int k = 0; k < VE; ++k) {
        const int64_t i = (int64_t)k * VB < n ? base + k * VB : (int64_t)f * A.nvox;
        rl[k] = A.r[i];
        pl[k] = A.p[i];
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < VE; ++k) {
        if ((int64_t)k * VB < n) {
            const float pf = (float)((double)rl[k] + beta * (double)pl[k]);
            A.p[base + k * VB] = pf;
            s += (double)pf * (double)pf;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) A.part[(int64_t)f * A.bpf + blockIdx.x] = s;
}

// ------------------------------------------------------- frame scalars --
struct ScalArgs {
    int64_t nvox;
    const double *part_vol;     // [nf * bpf]
    const double *part_beta;    // partials of ||r||^2 after the x, r update: [nf * bpf_beta]
    int64_t bpf_beta;
    const double *part_proj;    // [total tiles]
    const int64_t *tile_offset; // [nf + 1]
    double *scal;               // [SC_COUNT][nf]
    int32_t *iscal;             // [IS_COUNT][nf]
    const double *consts;       // inv_s2, tol, max_iter
    int nf, bpf;
};

// Fixed-order sum of a[lo, hi) by one workgroup: 8 independent loads in
// flight per thread, then the tail, then the workgroup reduction.
__device__ double frame_sum(const double *a, int64_t lo, int64_t hi)
{
    constexpr int U = 8;
    const int64_t step = blockDim.x;
    double s[U];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = 0.0;
    int64_t i = lo + threadIdx.x;
    for (; i + (U - 1) * step < hi; i += U * step) {
#pragma unroll
        for (int u = 0; u < U; ++u) s[u] += a[i + u * step];
    }
    for (; i < hi; i += step) s[0] += a[i];
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) t += s[u];
    return block_sum(t);
}

__device__ __forceinline__ double &S(ScalArgs &A, int slot, int f) { return A.scal[slot * A.nf + f]; }
__device__ __forceinline__ int32_t &I(ScalArgs &A, int slot, int f) { return A.iscal[slot * A.nf + f]; }

__global__ __launch_bounds__(VB) void k_red_setup(ScalArgs A, int what)
{
    const int f = blockIdx.x;
    const double s = frame_sum(A.part_vol, (int64_t)f * A.bpf, (int64_t)(f + 1) * A.bpf);
    if (threadIdx.x != 0) return;
    if (what == RW_BNORM) {
        S(A, SC_BNORM, f) = sqrt(s);
    } else if (what == RW_INIT) {
        const double bn = S(A, SC_BNORM, f);
        const double rel = bn > 0.0 ? sqrt(s) / bn : sqrt(s);
        S(A, SC_GAMMA, f) = s;
        S(A, SC_PP, f) = s;
        S(A, SC_REL, f) = rel;
        I(A, IS_ITERS, f) = 0;
        I(A, IS_STATUS, f) = 0;
        const bool done = (bn > 0.0 ? rel <= A.consts[1] : s == 0.0) || A.consts[2] < 1.0;
        I(A, IS_ACTIVE, f) = done ? 0 : 1;
    } else if (what == RW_TRUE) {
        const double bn = S(A, SC_BNORM, f);
        S(A, SC_TRUE, f) = bn > 0.0 ? sqrt(s) / bn : sqrt(s);
    } else if (what == RW_REPLACE) {
        // the recursive residual replaced by the FP64 one, CG restarted from it (p = r)
        const double bn = S(A, SC_BNORM, f);
        const double rel = bn > 0.0 ? sqrt(s) / bn : sqrt(s);
        S(A, SC_GAMMA, f) = s;
        S(A, SC_PP, f) = s;
        S(A, SC_REL, f) = rel;
        S(A, SC_TRUE, f) = rel;
        const bool done = (bn > 0.0 ? rel <= A.consts[3] : s == 0.0) || I(A, IS_ITERS, f) >= (int)A.consts[2];
        if (I(A, IS_STATUS, f) != MSF_EBREAKDOWN) I(A, IS_ACTIVE, f) = done ? 0 : 1;
    } else if (what == RW_DIAG) {
        // mean of A^T Lambda A 1 over the frame's voxels, plus the 1/sigma^2 of H
        S(A, SC_DIAG, f) = s / (double)A.nvox + A.consts[0];
    } else {
        // learned start: keep it where it is finite and beats the residual of v
        S(A, SC_GCNN, f) = s;
        const bool keep = isfinite(s) && s < S(A, SC_GAMMA, f);
        I(A, IS_CNN, f) = keep ? 1 : 0;
        if (keep) {
            const double bn = S(A, SC_BNORM, f);
            const double rel = bn > 0.0 ? sqrt(s) / bn : sqrt(s);
            S(A, SC_GAMMA, f) = s;
            S(A, SC_PP, f) = s;
            S(A, SC_REL, f) = rel;
            const bool done = (bn > 0.0 ? rel <= A.consts[1] : s == 0.0) || A.consts[2] < 1.0;
            I(A, IS_ACTIVE, f) = done ? 0 : 1;
        }
    }
}

__global__ __launch_bounds__(VB) void k_red_alpha(ScalArgs A)
{
    const int f = blockIdx.x;
    if (!I(A, IS_ACTIVE, f)) return;
    const double wlw = frame_sum(A.part_proj, A.tile_offset[f], A.tile_offset[f + 1]);
    const double pp = frame_sum(A.part_vol, (int64_t)f * A.bpf, (int64_t)(f + 1) * A.bpf);
    if (threadIdx.x != 0) return;
    const double pq = wlw + pp * A.consts[0];
    S(A, SC_PP, f) = pp;
    S(A, SC_PQ, f) = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
        I(A, IS_STATUS, f) = MSF_EBREAKDOWN;
        I(A, IS_ACTIVE, f) = 0;
        S(A, SC_ALPHA, f) = 0.0;
        return;
    }
    S(A, SC_ALPHA, f) = S(A, SC_GAMMA, f) / pq;
}

__global__ __launch_bounds__(VB) void k_red_beta(ScalArgs A)
{
    const int f = blockIdx.x;
    if (!I(A, IS_ACTIVE, f)) return;
    const double g = frame_sum(A.part_beta, (int64_t)f * A.bpf_beta, (int64_t)(f + 1) * A.bpf_beta);
    if (threadIdx.x != 0) return;
    const double bn = S(A, SC_BNORM, f);
    const double rel = bn > 0.0 ? sqrt(g) / bn : sqrt(g);
    const int it = I(A, IS_ITERS, f) + 1;
    I(A, IS_ITERS, f) = it;
    S(A, SC_REL, f) = rel;
    S(A, SC_BETA, f) = g / S(A, SC_GAMMA, f);
    S(A, SC_GAMMA, f) = g;
    if (!isfinite(g)) {
        I(A, IS_STATUS, f) = MSF_EBREAKDOWN;
        I(A, IS_ACTIVE, f) = 0;
    } else if ((bn > 0.0 ? rel <= A.consts[1] : g == 0.0) || it >= (int)A.consts[2]) {
        I(A, IS_ACTIVE, f) = 0;
    }
}

VolArgs vol_args(msf_plan &P, bool with_active)
{
    VolArgs A;
    A.x = P.x; A.r = P.r; A.p = P.p; A.bp = P.bp; A.x64 = P.x64; A.vin = P.vin;
    A.part = P.part_vol;
    A.scal = P.scal;
    A.active = with_active ? P.iscal + IS_ACTIVE * P.nf : nullptr;
    A.consts = P.consts;
    A.nvox = P.nvox;
    A.nf = P.nf;
    A.bpf = (int)P.vol_blocks_per_frame;
    return A;
}

ScalArgs scal_args(msf_plan &P, bool fused = false)
{
    ScalArgs A;
    A.nvox = P.nvox;
    A.part_vol = P.part_vol;
    A.part_beta = fused ? P.part_g : P.part_vol;
    A.bpf_beta = fused ? P.part_g_per_frame : P.vol_blocks_per_frame;
    A.part_proj = P.part_proj;
    A.tile_offset = P.d_tile_offset;
    A.scal = P.scal;
    A.iscal = P.iscal;
    A.consts = P.consts;
    A.nf = P.nf;
    A.bpf = (int)P.vol_blocks_per_frame;
    return A;
}

}  // namespace

hipError_t launch_transpose(const float *in, float *out, int64_t B, int R, int C, int check, int32_t *flags,
                            hipStream_t s)
{
    if (B == 0 || R == 0 || C == 0) return hipSuccess;
    dim3 grid((C + 31) / 32, (R + 31) / 32, (unsigned)B), block(32, 8);
    hipLaunchKernelGGL(k_transpose, grid, block, 0, s, in, out, R, C, check, flags);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_d(double *p, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_d, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_d2f(const double *src, float *dst, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_d2f, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_sino_mul_scaled(const float *a, const float *b, const float *scale, int64_t per_view, float *out,
                                  int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mul_scaled, dim3(grid_for(n)), dim3(256), 0, s, a, b, scale, per_view, out, n);
    return hipGetLastError();
}

hipError_t launch_sino_mul(const float *a, const float *b, float *out, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mul, dim3(grid_for(n)), dim3(256), 0, s, a, b, out, n);
    return hipGetLastError();
}

static dim3 vol_grid(const msf_plan &P) { return dim3((unsigned)P.vol_blocks_per_frame, (unsigned)P.nf); }

hipError_t launch_vol_bnorm(msf_plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_vol_bnorm, vol_grid(P), dim3(VB), 0, s, vol_args(P, false));
    return hipGetLastError();
}

hipError_t launch_vol_init_residual(msf_plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_vol_residual, vol_grid(P), dim3(VB), 0, s, vol_args(P, false), 1);
    return hipGetLastError();
}

hipError_t launch_vol_true_residual(msf_plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_vol_residual, vol_grid(P), dim3(VB), 0, s, vol_args(P, false), 0);
    return hipGetLastError();
}

hipError_t launch_vol_sum_bp(msf_plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_vol_sum_bp, vol_grid(P), dim3(VB), 0, s, vol_args(P, false));
    return hipGetLastError();
}

hipError_t launch_scale_feature(msf_plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_feature, vol_grid(P), dim3(VB), 0, s, vol_args(P, false));
    return hipGetLastError();
}

hipError_t launch_vol_residual_p(msf_plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_vol_residual, vol_grid(P), dim3(VB), 0, s, vol_args(P, false), 2);
    return hipGetLastError();
}

hipError_t launch_fold_correction(msf_plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold, vol_grid(P), dim3(VB), 0, s, vol_args(P, false));
    return hipGetLastError();
}

hipError_t launch_vol_residual64(msf_plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_vol_residual64, vol_grid(P), dim3(VB), 0, s, vol_args(P, false));
    return hipGetLastError();
}

hipError_t launch_vol_select(msf_plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_vol_select, vol_grid(P), dim3(VB), 0, s, vol_args(P, false), P.iscal + IS_CNN * P.nf);
    return hipGetLastError();
}

hipError_t launch_scalar_reduce(msf_plan &P, int what, hipStream_t s)
{
    hipLaunchKernelGGL(k_red_setup, dim3(P.nf), dim3(VB), 0, s, scal_args(P), what);
    return hipGetLastError();
}

hipError_t launch_cg_step(msf_plan &P, hipStream_t s, hipEvent_t *ev)
{
    hipError_t e;
    // the voxel-driven adjoint finishes the x, r update in its epilogue
    const bool fused = P.tiles.back_mode != 0;
    if (ev && (e = hipEventRecordWithFlags(ev[0], s, hipEventRecordExternal)) != hipSuccess) return e;
    if ((e = launch_forward(P, PM_WEIGHTED, P.p, nullptr, P.sz, true, s)) != hipSuccess) return e;
    if (ev && (e = hipEventRecordWithFlags(ev[1], s, hipEventRecordExternal)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_red_alpha, dim3(P.nf), dim3(VB), 0, s, scal_args(P));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecordWithFlags(ev[2], s, hipEventRecordExternal)) != hipSuccess) return e;
    if (fused) {
        if ((e = launch_back_gather_update(P, s)) != hipSuccess) return e;
        if (ev && (e = hipEventRecordWithFlags(ev[3], s, hipEventRecordExternal)) != hipSuccess) return e;
    } else {
        if ((e = launch_back(P, P.sz, P.bp, true, s)) != hipSuccess) return e;
        if (ev && (e = hipEventRecordWithFlags(ev[3], s, hipEventRecordExternal)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_update_xr, vol_grid(P), dim3(VB), 0, s, vol_args(P, true));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_red_beta, dim3(P.nf), dim3(VB), 0, s, scal_args(P, fused));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_update_p, vol_grid(P), dim3(VB), 0, s, vol_args(P, true));
    return hipGetLastError();
}

int64_t vol_chunk() { return VCHUNK; }
