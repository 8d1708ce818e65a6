// Multi-agent consensus equilibrium (paper Sec. III) around the batched
// proximal map: Algorithm 1, the partial-update Mann iteration
//     X <- F~(W; X);   Z <- G(2X - W);   W <- W + 2 rho (Z - X),
// with F~ = [L~(W_0; X_0), H_1(W_1), ..., H_K(W_K)] (eq. (13)),
// G the weighted averaging of eqs. (8), (9), and the output X_0.
//
// L~ is msf_prox_solve on W_0 started from the previous X_0: to the tolerance
// (full proximal map) or for a fixed number of CG steps (the partial update
// the paper uses with three coordinate-descent sweeps).  The prior agents are
// the paper's multi-slice fusion denoisers H_xy,t, H_yz,t, H_zx,t (Sec. IV):
// one trained 2.5D CNN (cnn.hip) applied to every 2D slice of the xy, yz or
// zx planes with the same slice at time points t-2 .. t+2 as its channels;
// or stand-ins that are true proximal maps, for which the equilibrium has a
// closed form: symmetric plane-wise Gaussian smoothers in the xy, yz and zx
// planes (eigenvalues in (0, 1]), or the ridge shrinkage x / (1 + lambda
// sigma^2), the proximal map of (lambda/2) ||x||^2.
//
// Volumes are kept in the public layout [frame][nz][ny][nx].  The averaging
// and the Mann update are one fused pass over the 2 (K + 1) state volumes.
#include "msf_internal.h"

#include <chrono>
#include <cmath>
#include <vector>

namespace {

constexpr int GR = 3;   // Gaussian radius in voxels (7 taps)

struct Blur1D {
    const float *in;
    float *out;
    int64_t n_frames;
    int nx, ny, nz;
    int axis;             // 0 = x, 1 = y, 2 = z
    float w[2 * GR + 1];
};

// out = symmetric 1D Gaussian along one axis, zero outside the volume
__global__ void k_blur1d(const Blur1D B)
{
    const int64_t total = B.n_frames * (int64_t)B.nz * B.ny * B.nx;
    const int64_t stride = B.axis == 0 ? 1 : (B.axis == 1 ? (int64_t)B.nx : (int64_t)B.nx * B.ny);
    const int len = B.axis == 0 ? B.nx : (B.axis == 1 ? B.ny : B.nz);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)((i / stride) % len);
        float s = 0.0f;
#pragma unroll
        for (int t = -GR; t <= GR; ++t) {
            const int cc = c + t;
            if (cc >= 0 && cc < len) s = fmaf(B.w[t + GR], B.in[i + t * stride], s);
        }
        B.out[i] = s;
    }
}

__global__ void k_scale(const float *__restrict__ in, float *__restrict__ out, int64_t n, float a)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a * in[i];
}

struct MannArgs {
    float *W[4];
    const float *X[4];
    int K;                // prior agents (components 1..K)
    float w0, wk;         // averaging weights: 1/(1+beta), beta/((1+beta) K)
    float two_rho;
    int64_t n;
};

// zbar = w0 (2 X_0 - W_0) + wk sum_k (2 X_k - W_k);  W_k += 2 rho (zbar - X_k)
__global__ void k_mann(const MannArgs A)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * blockDim.x) {
        float x[4], w[4];
        for (int k = 0; k <= A.K; ++k) {
            x[k] = A.X[k][i];
            w[k] = A.W[k][i];
        }
        float zbar = A.w0 * (2.0f * x[0] - w[0]);
        float pri = 0.0f;
        for (int k = 1; k <= A.K; ++k) pri += 2.0f * x[k] - w[k];
        zbar = fmaf(A.wk, pri, zbar);
        for (int k = 0; k <= A.K; ++k) A.W[k][i] = fmaf(A.two_rho, zbar - x[k], w[k]);
    }
}

unsigned grid_n(int64_t n)
{
    int64_t g = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

#define MCHK(expr)                                           \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

}  // namespace

extern "C" {

void msf_mace_opts_default(msf_mace_opts *o)
{
    if (!o) return;
    o->n_iter = 10;
    o->prior = MSF_PRIOR_PLANE_GAUSS;
    o->partial_iters = 0;
    o->max_iter = 2000;
    o->beta = 1.0;
    o->rho = 0.5;
    o->prior_param = 1.0;
    o->tol = 1e-6;
    o->cnn = nullptr;
    o->prior_cnn = nullptr;
}

msf_status msf_mace_run(msf_plan *P, const float *x_init, const float *y, const float *lam, double sigma,
                        const msf_mace_opts *opts, float *x_out, msf_mace_stats *stats, void *stream)
{
    set_error("");
    const auto t0 = std::chrono::steady_clock::now();
    if (!P || !y || !lam || !x_out || !opts) { set_error("null argument"); return MSF_EINVAL; }
    const msf_mace_opts &o = *opts;
    if (!(sigma > 0.0 && std::isfinite(sigma)) || o.n_iter < 0 || !(o.beta > 0.0) || !(o.rho > 0.0 && o.rho < 1.0) ||
        !(o.prior_param > 0.0) || o.partial_iters < 0 ||
        (o.prior != MSF_PRIOR_PLANE_GAUSS && o.prior != MSF_PRIOR_RIDGE && o.prior != MSF_PRIOR_CNN) ||
        (o.prior == MSF_PRIOR_CNN && (!o.prior_cnn || cnn_kind(o.prior_cnn) != MSF_CNN_DENOISER))) {
        set_error("invalid MACE options (sigma > 0, n_iter >= 0, beta > 0, 0 < rho < 1, prior_param > 0, "
                  "a known prior, a denoiser network for MSF_PRIOR_CNN)");
        return MSF_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int K = 3;
    const int64_t n = P->nvox_total;
    std::vector<float *> W(K + 1, nullptr), X(K + 1, nullptr);
    float *tmp = nullptr, *sa = nullptr, *sb = nullptr;
    auto cleanup = [&]() {
        for (float *q : W) if (q) (void)hipFree(q);
        for (float *q : X) if (q) (void)hipFree(q);
        if (tmp) (void)hipFree(tmp);
        if (sa) (void)hipFree(sa);
        if (sb) (void)hipFree(sb);
    };
    hipError_t e = hipSuccess;
    for (int k = 0; k <= K && e == hipSuccess; ++k) {
        e = hipMalloc((void **)&W[k], sizeof(float) * std::max<int64_t>(n, 1));
        if (e == hipSuccess) e = hipMalloc((void **)&X[k], sizeof(float) * std::max<int64_t>(n, 1));
    }
    if (e == hipSuccess) e = hipMalloc((void **)&tmp, sizeof(float) * std::max<int64_t>(n, 1));
    if (e == hipSuccess && o.prior == MSF_PRIOR_CNN) {   // plane sequences of the yz and zx agents
        e = hipMalloc((void **)&sa, sizeof(float) * std::max<int64_t>(n, 1));
        if (e == hipSuccess) e = hipMalloc((void **)&sb, sizeof(float) * std::max<int64_t>(n, 1));
    }
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "MACE state allocation"); }
    // X = W = [x_init; ...] (zero when x_init is NULL, the paper's initial condition)
    for (int k = 0; k <= K && e == hipSuccess; ++k) {
        e = x_init ? launch_copy(W[k], x_init, n, s) : launch_fill(W[k], n, 0.0f, s);
        if (e == hipSuccess) e = launch_copy(X[k], W[k], n, s);
    }
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "MACE init"); }

    Blur1D bl{};
    bl.n_frames = P->nf; bl.nx = P->nx; bl.ny = P->ny; bl.nz = P->nz;
    double wsum = 0.0;
    for (int t = -GR; t <= GR; ++t) wsum += std::exp(-0.5 * t * t / (o.prior_param * o.prior_param));
    for (int t = -GR; t <= GR; ++t)
        bl.w[t + GR] = (float)(std::exp(-0.5 * t * t / (o.prior_param * o.prior_param)) / wsum);
    const int planes[3][2] = {{0, 1}, {1, 2}, {2, 0}};   // xy, yz, zx

    int64_t cg_total = 0;
    msf_status worst = MSF_OK;
    for (int it = 0; it < o.n_iter; ++it) {
        // data-term agent: L~(W_0; X_0), started from the previous X_0
        msf_solve_opts so;
        msf_solve_opts_default(&so);
        so.x0_mode = o.cnn && it == 0 ? MSF_X0_CNN : MSF_X0_USER;
        so.x0 = X[0];
        so.cnn = o.cnn;
        so.check_every = 16;
        if (o.partial_iters > 0) {
            so.tol = 0.0;
            so.max_iter = o.partial_iters;
        } else {
            so.tol = o.tol;
            so.max_iter = o.max_iter;
        }
        std::vector<int32_t> iters(P->nf, 0);
        msf_solve_stats ss{};
        ss.iters = iters.data();
        msf_status st = msf_prox_solve(P, W[0], y, lam, sigma, &so, X[0], &ss, stream);
        if (st < 0) { cleanup(); return st; }
        if (st == MSF_NOT_CONVERGED && o.partial_iters == 0) worst = MSF_NOT_CONVERGED;
        for (int32_t v : iters) cg_total += v;
        if (stats && stats->cg_iters && it < stats->capacity) {
            int64_t tot = 0;
            for (int32_t v : iters) tot += v;
            stats->cg_iters[it] = tot;
        }
        // prior agents
        for (int k = 1; k <= K; ++k) {
            if (o.prior == MSF_PRIOR_CNN) {
                // H_k: the 2.5D denoiser on the slices of plane k (Sec. IV)
                e = denoise25_internal(const_cast<msf_cnn *>(o.prior_cnn), W[k], P->nf, P->nz, P->ny, P->nx, k, X[k],
                                       sa, sb, s);
                if (e != hipSuccess) { cleanup(); return hip_fail(e, "CNN prior agent"); }
                continue;
            }
            if (o.prior == MSF_PRIOR_RIDGE) {
                hipLaunchKernelGGL(k_scale, dim3(grid_n(n)), dim3(256), 0, s, W[k], X[k], n,
                                   (float)(1.0 / (1.0 + o.prior_param * sigma * sigma)));
            } else {
                bl.in = W[k]; bl.out = tmp; bl.axis = planes[k - 1][0];
                hipLaunchKernelGGL(k_blur1d, dim3(grid_n(n)), dim3(256), 0, s, bl);
                bl.in = tmp; bl.out = X[k]; bl.axis = planes[k - 1][1];
                hipLaunchKernelGGL(k_blur1d, dim3(grid_n(n)), dim3(256), 0, s, bl);
            }
            if ((e = hipGetLastError()) != hipSuccess) { cleanup(); return hip_fail(e, "prior agent"); }
        }
        // Z <- G(2X - W); W <- W + 2 rho (Z - X)
        MannArgs M{};
        for (int k = 0; k <= K; ++k) {
            M.W[k] = W[k];
            M.X[k] = X[k];
        }
        M.K = K;
        M.w0 = (float)(1.0 / (1.0 + o.beta));
        M.wk = (float)(o.beta / ((1.0 + o.beta) * K));
        M.two_rho = (float)(2.0 * o.rho);
        M.n = n;
        hipLaunchKernelGGL(k_mann, dim3(grid_n(n)), dim3(256), 0, s, M);
        if ((e = hipGetLastError()) != hipSuccess) { cleanup(); return hip_fail(e, "Mann update"); }
    }
    e = launch_copy(x_out, X[0], n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) return hip_fail(e, "MACE output");
    if (stats) {
        stats->cg_total = cg_total;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return worst;
}

}  // extern "C"
