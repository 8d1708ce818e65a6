// Blind fixture correction (paper Appendix A, algorithm "Blind fixture
// correction"): remove from the measurement the smooth projection of fixtures
// outside the field of view.  From a reconstruction x:
//     x_m = cylinder mask of x;  e = y - A x_m;  p = blur(e);
//     c = argmin_c ||e - c p||^2 = <e, p> / <p, p>;  y_corr = y - c p,
// one c per time frame.  The projection uses the plan's forward projector;
// the blur is a separable Gaussian over the detector's u and v within each
// view (values outside the detector taken as zero), evaluated in FP64 from
// FP32 data; the inner products are FP64, summed in a fixed order.
//
// Layouts are the plan's internal ones: volume [frame][ny][nx][nz], sinogram
// [view][nu][nv].
#include "msf_internal.h"

#include <cmath>
#include <vector>

namespace {

constexpr int MAX_R = 64;   // blur radius limit in detector pixels

struct Taps {
    double w[2 * MAX_R + 1];
    int r;
};

// zero the voxels whose centre is farther than sqrt(r2) from the rotation axis
__global__ void k_cyl_mask(float *__restrict__ vol, int64_t nvox_total, int nx, int ny, int nz, double r2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nvox_total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / nz;              // (frame, iy, ix) column
        const int ix = (int)(c % nx);
        const int iy = (int)((c / nx) % ny);
        const double dx = ix - 0.5 * (nx - 1), dy = iy - 0.5 * (ny - 1);
        if (dx * dx + dy * dy > r2) vol[i] = 0.0f;
    }
}

// a = b - a
__global__ void k_rsub(float *__restrict__ a, const float *__restrict__ b, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = b[i] - a[i];
}

// 1D Gaussian along v (stride 1, length nv) or u (stride nv, length nu) of every view
__global__ void k_blur(const float *__restrict__ in, float *__restrict__ out, int64_t n, int nu, int nv, int along_u,
                       const Taps T)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int iv = (int)(i % nv);
        const int iu = (int)((i / nv) % nu);
        const int c = along_u ? iu : iv, len = along_u ? nu : nv;
        const int64_t stride = along_u ? nv : 1;
        const int lo = max(-T.r, -c), hi = min(T.r, len - 1 - c);
        double s = 0.0;
        for (int t = lo; t <= hi; ++t) s += T.w[t + T.r] * (double)in[i + t * stride];
        out[i] = (float)s;
    }
}

// per view: <e, p> and <p, p> in FP64 (one workgroup per view, fixed order)
__global__ __launch_bounds__(256) void k_view_dots(const float *__restrict__ e, const float *__restrict__ p,
                                                   int64_t per_view, double *__restrict__ out)
{
    const int64_t v = blockIdx.x;
    const float *ev = e + v * per_view, *pv = p + v * per_view;
    double ep = 0.0, pp = 0.0;
    for (int64_t i = threadIdx.x; i < per_view; i += blockDim.x) {
        const double a = ev[i], b = pv[i];
        ep += a * b;
        pp += b * b;
    }
    __shared__ double red[2][4];
    for (int o = 32; o > 0; o >>= 1) {
        ep += __shfl_xor(ep, o, 64);
        pp += __shfl_xor(pp, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x / 64] = ep;
        red[1][threadIdx.x / 64] = pp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        out[2 * v] = a;
        out[2 * v + 1] = b;
    }
}

// per frame: c = sum <e, p> / sum <p, p> over its views (in view order)
__global__ void k_frame_fit(const double *__restrict__ dots, const int64_t *__restrict__ view_offset, int nf,
                            double *__restrict__ c)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    double ep = 0.0, pp = 0.0;
    for (int64_t v = view_offset[f]; v < view_offset[f + 1]; ++v) {
        ep += dots[2 * v];
        pp += dots[2 * v + 1];
    }
    c[f] = pp > 0.0 ? ep / pp : 0.0;
}

// out = y - c[frame of the element's view] p
__global__ void k_apply(const float *__restrict__ y, const float *__restrict__ p, const double *__restrict__ c,
                        const int64_t *__restrict__ view_offset, int nf, int64_t per_view, int64_t n,
                        float *__restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = i / per_view;
        int lo = 0, hi = nf;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (view_offset[mid] <= v) lo = mid;
            else hi = mid;
        }
        out[i] = (float)((double)y[i] - c[lo] * (double)p[i]);
    }
}

unsigned grid_of(int64_t n)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
}

#define FCHK(expr)                                           \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) {                              \
            release();                                       \
            return hip_fail(e_, #expr);                      \
        }                                                    \
    } while (0)

}  // namespace

extern "C" msf_status msf_fixture_correct(msf_plan *P, const float *x, const float *y, double mask_radius,
                                          double blur_std, float *y_corr, double *c_out, void *stream)
{
    set_error("");
    if (!P || !x || !y || !y_corr) { set_error("null argument"); return MSF_EINVAL; }
    if (!(mask_radius > 0.0 && std::isfinite(mask_radius))) { set_error("mask_radius must be > 0"); return MSF_EINVAL; }
    const int r = (int)std::ceil(3.0 * blur_std);
    if (!(blur_std > 0.0) || !std::isfinite(blur_std) || r > MAX_R) {
        set_error("blur_std must be > 0 with 3 std <= 64 pixels");
        return MSF_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    Taps T{};
    T.r = r;
    double sum = 0.0;
    for (int t = -r; t <= r; ++t) sum += std::exp(-0.5 * t * t / (blur_std * blur_std));
    for (int t = -r; t <= r; ++t) T.w[t + r] = std::exp(-0.5 * t * t / (blur_std * blur_std)) / sum;

    const int64_t nm = P->nmeas_total, per_view = (int64_t)P->nu * P->nv;
    float *ptmp = nullptr;
    double *dots = nullptr, *cdev = nullptr;
    auto release = [&]() {
        if (ptmp) (void)hipFree(ptmp);
        if (dots) (void)hipFree(dots);
        if (cdev) (void)hipFree(cdev);
    };
    FCHK(hipMalloc((void **)&ptmp, sizeof(float) * std::max<int64_t>(nm, 1)));
    FCHK(hipMalloc((void **)&dots, sizeof(double) * 2 * std::max<int64_t>(P->n_views, 1)));
    FCHK(hipMalloc((void **)&cdev, sizeof(double) * P->nf));

    // x_m (internal layout) and A x_m
    FCHK(vol_to_internal(*P, x, P->p, 0, nullptr, s));
    hipLaunchKernelGGL(k_cyl_mask, dim3(grid_of(P->nvox_total)), dim3(256), 0, s, P->p, P->nvox_total, P->nx, P->ny,
                       P->nz, mask_radius * mask_radius);
    FCHK(hipGetLastError());
    FCHK(launch_fill(P->sz, nm, 0.0f, s));
    FCHK(launch_forward(*P, PM_PLAIN, P->p, nullptr, P->sz, false, s));
    // e = y - A x_m  (in sz; y stays in sy)
    FCHK(sino_to_internal(*P, y, P->sy, 0, nullptr, s));
    hipLaunchKernelGGL(k_rsub, dim3(grid_of(nm)), dim3(256), 0, s, P->sz, P->sy, nm);
    FCHK(hipGetLastError());
    // p = blur(e): along v into slam, then along u into ptmp
    if (nm > 0) {
        hipLaunchKernelGGL(k_blur, dim3(grid_of(nm)), dim3(256), 0, s, P->sz, P->slam, nm, P->nu, P->nv, 0, T);
        hipLaunchKernelGGL(k_blur, dim3(grid_of(nm)), dim3(256), 0, s, P->slam, ptmp, nm, P->nu, P->nv, 1, T);
        FCHK(hipGetLastError());
        hipLaunchKernelGGL(k_view_dots, dim3((unsigned)P->n_views), dim3(256), 0, s, P->sz, ptmp, per_view, dots);
        FCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_frame_fit, dim3((P->nf + 63) / 64), dim3(64), 0, s, dots, P->d_view_offset, P->nf, cdev);
    FCHK(hipGetLastError());
    if (nm > 0) {
        hipLaunchKernelGGL(k_apply, dim3(grid_of(nm)), dim3(256), 0, s, P->sy, ptmp, cdev, P->d_view_offset, P->nf,
                           per_view, nm, P->sz);
        FCHK(hipGetLastError());
    }
    FCHK(sino_to_public(*P, P->sz, y_corr, s));
    std::vector<double> hc(P->nf, 0.0);
    FCHK(hipMemcpyAsync(hc.data(), cdev, sizeof(double) * P->nf, hipMemcpyDeviceToHost, s));
    FCHK(hipStreamSynchronize(s));
    release();
    if (c_out)
        for (int f = 0; f < P->nf; ++f) c_out[f] = hc[f];
    return MSF_OK;
}
