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
#include <mutex>
#include <string>
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

// Scratch of the allocation-free entry point: the blurred sinogram p, the
// per-view inner products and the per-frame fits, in one file-scope device
// array.  Each GPU the library runs on holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol): it asks each device for the array's
// address once and passes that.
constexpr size_t SCRATCH_BYTES = (size_t)MSF_FIXTURE_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Address of `scratch` on the current device (looked up on the first call per device).
msf_status scratch_on_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("device index beyond the scratch table");
        return MSF_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MSF_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Blur taps of std blur_std over 2 ceil(3 std) + 1 pixels, normalised.
msf_status make_taps(double blur_std, Taps &T)
{
    const int r = (int)std::ceil(3.0 * blur_std);
    if (!(blur_std > 0.0) || !std::isfinite(blur_std) || r > MAX_R) {
        set_error("blur_std must be > 0 with 3 std <= 64 pixels");
        return MSF_EINVAL;
    }
    T = Taps{};
    T.r = r;
    double sum = 0.0;
    for (int t = -r; t <= r; ++t) sum += std::exp(-0.5 * t * t / (blur_std * blur_std));
    for (int t = -r; t <= r; ++t) T.w[t + r] = std::exp(-0.5 * t * t / (blur_std * blur_std)) / sum;
    return MSF_OK;
}

#define RCHK(expr)                                           \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

// The correction on the stream, with its scratch given: ptmp [n_meas] FP32,
// dots [2 n_views] FP64, cdev [n_frames] FP64 (every element is written
// before it is read).  Leaves c in cdev; nothing is synchronised.
msf_status run_correction(msf_plan *P, const float *x, const float *y, double mask_radius, const Taps &T,
                          float *y_corr, float *ptmp, double *dots, double *cdev, hipStream_t s)
{
    const int64_t nm = P->nmeas_total, per_view = (int64_t)P->nu * P->nv;
    // x_m (internal layout) and A x_m
    RCHK(vol_to_internal(*P, x, P->p, 0, nullptr, s));
    hipLaunchKernelGGL(k_cyl_mask, dim3(grid_of(P->nvox_total)), dim3(256), 0, s, P->p, P->nvox_total, P->nx, P->ny,
                       P->nz, mask_radius * mask_radius);
    RCHK(hipGetLastError());
    RCHK(launch_fill(P->sz, nm, 0.0f, s));
    RCHK(launch_forward(*P, PM_PLAIN, P->p, nullptr, P->sz, false, s));
    // e = y - A x_m  (in sz; y stays in sy)
    RCHK(sino_to_internal(*P, y, P->sy, 0, nullptr, s));
    hipLaunchKernelGGL(k_rsub, dim3(grid_of(nm)), dim3(256), 0, s, P->sz, P->sy, nm);
    RCHK(hipGetLastError());
    // p = blur(e): along v into slam, then along u into ptmp
    if (nm > 0) {
        hipLaunchKernelGGL(k_blur, dim3(grid_of(nm)), dim3(256), 0, s, P->sz, P->slam, nm, P->nu, P->nv, 0, T);
        hipLaunchKernelGGL(k_blur, dim3(grid_of(nm)), dim3(256), 0, s, P->slam, ptmp, nm, P->nu, P->nv, 1, T);
        RCHK(hipGetLastError());
        hipLaunchKernelGGL(k_view_dots, dim3((unsigned)P->n_views), dim3(256), 0, s, P->sz, ptmp, per_view, dots);
        RCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_frame_fit, dim3((P->nf + 63) / 64), dim3(64), 0, s, dots, P->d_view_offset, P->nf, cdev);
    RCHK(hipGetLastError());
    if (nm > 0) {
        hipLaunchKernelGGL(k_apply, dim3(grid_of(nm)), dim3(256), 0, s, P->sy, ptmp, cdev, P->d_view_offset, P->nf,
                           per_view, nm, P->sz);
        RCHK(hipGetLastError());
    }
    RCHK(sino_to_public(*P, P->sz, y_corr, s));
    return MSF_OK;
}

}  // namespace

extern "C" msf_status msf_fixture_correct(msf_plan *P, const float *x, const float *y, double mask_radius,
                                          double blur_std, float *y_corr, double *c_out, void *stream)
{
    set_error("");
    if (!P || !x || !y || !y_corr) { set_error("null argument"); return MSF_EINVAL; }
    if (!(mask_radius > 0.0 && std::isfinite(mask_radius))) { set_error("mask_radius must be > 0"); return MSF_EINVAL; }
    Taps T;
    msf_status st = make_taps(blur_std, T);
    if (st != MSF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nm = P->nmeas_total;
    float *ptmp = nullptr;
    double *dots = nullptr, *cdev = nullptr;
    auto release = [&]() {
        if (ptmp) (void)hipFree(ptmp);
        if (dots) (void)hipFree(dots);
        if (cdev) (void)hipFree(cdev);
    };
    hipError_t e = hipMalloc((void **)&ptmp, sizeof(float) * std::max<int64_t>(nm, 1));
    if (e == hipSuccess) e = hipMalloc((void **)&dots, sizeof(double) * 2 * std::max<int64_t>(P->n_views, 1));
    if (e == hipSuccess) e = hipMalloc((void **)&cdev, sizeof(double) * P->nf);
    if (e != hipSuccess) {
        release();
        return hip_fail(e, "hipMalloc fixture buffers");
    }
    st = run_correction(P, x, y, mask_radius, T, y_corr, ptmp, dots, cdev, s);
    std::vector<double> hc(P->nf, 0.0);
    if (st == MSF_OK) {
        e = hipMemcpyAsync(hc.data(), cdev, sizeof(double) * P->nf, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "fixture result");
    }
    release();
    if (st == MSF_OK && c_out)
        for (int f = 0; f < P->nf; ++f) c_out[f] = hc[f];
    return st;
}

extern "C" msf_status msf_fixture_correct_noalloc(msf_plan *P, const float *x, const float *y, double mask_radius,
                                                  double blur_std, float *y_corr, double *c_out, void *stream)
{
    set_error("");
    if (!P || !x || !y || !y_corr) { set_error("null argument"); return MSF_EINVAL; }
    if (!(mask_radius > 0.0 && std::isfinite(mask_radius))) { set_error("mask_radius must be > 0"); return MSF_EINVAL; }
    Taps T;
    msf_status st = make_taps(blur_std, T);
    if (st != MSF_OK) return st;
    // scratch layout: dots [2 n_views] FP64 | cdev [n_frames] FP64 | ptmp [n_meas] FP32, each 256-byte aligned
    const size_t off_c = align256(sizeof(double) * 2 * (size_t)P->n_views);
    const size_t off_p = off_c + align256(sizeof(double) * (size_t)P->nf);
    const size_t need = off_p + sizeof(float) * (size_t)P->nmeas_total;
    if (need > SCRATCH_BYTES) {
        set_error("msf_fixture_correct_noalloc: this geometry needs " + std::to_string(need) +
                  " bytes of scratch, more than its " + std::to_string(SCRATCH_BYTES) +
                  "-byte limit (use msf_fixture_correct)");
        return MSF_EINVAL;
    }
    void *base = nullptr;
    if ((st = scratch_on_current_device(&base)) != MSF_OK) return st;
    char *b = (char *)base;
    double *dots = (double *)b, *cdev = (double *)(b + off_c);
    float *ptmp = (float *)(b + off_p);
    hipStream_t s = (hipStream_t)stream;
    if ((st = run_correction(P, x, y, mask_radius, T, y_corr, ptmp, dots, cdev, s)) != MSF_OK) return st;
    // c through the plan's pinned staging buffer (sized for more than n_frames doubles at creation)
    double *hc = (double *)P->host_stage;
    RCHK(hipMemcpyAsync(hc, cdev, sizeof(double) * P->nf, hipMemcpyDeviceToHost, s));
    RCHK(hipStreamSynchronize(s));
    if (c_out)
        for (int f = 0; f < P->nf; ++f) c_out[f] = hc[f];
    return MSF_OK;
}
