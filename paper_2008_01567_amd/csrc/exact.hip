// FP64 residual of the proximal-map system for iterative refinement
// (paper Sec. III, eq. (4): r = b - H x with H = A^T Lambda A + sigma^-2 I,
// b = A^T Lambda y + sigma^-2 v, i.e. r = A^T Lambda (y - A x) + (v - x) / sigma^2).
//
// The CG steps run on the FP32 projector, whose lengths are FP32 differences
// of rounded plane crossings and whose sinogram intermediate is FP32.  On
// stiff systems (the paper's weights Lambda = c exp(-A x0)) the error of the
// solution is thousands of times its relative residual, so those FP32
// roundings put a floor under the error that no number of CG steps removes.
// Mixed-precision iterative refinement removes that floor: the iterate is
// kept in FP64, its residual is computed here with FP64 lengths, an FP64
// sinogram and FP64 sums, and the FP32 CG only solves for the correction of
// the iterate, to a modest accuracy, before the correction is added in FP64
// and the residual recomputed.
//
// One thread per ray.  The ray is the segment from the source to the pixel
// centre, S + t d, t in [0, 1]; it is clipped to the volume box and cut at
// every x, y and z voxel plane (the three plane families merged on the fly,
// Siddon 1985 / Jacobs et al. 1998), each piece credited to the voxel that
// holds its midpoint (half-open voxels), with length (t1 - t0) |d| in FP64.
// The adjoint runs the same traversal and adds length * value into an FP64
// volume with hardware FP64 atomics.  It is slow next to the FP32 kernels
// and is used once per refinement, not once per CG step.
//
// Layouts are the plan's internal ones: volume [frame][ny][nx][nz], sinogram
// [view][nu][nv].
#include "msf_internal.h"
#include "exact_traverse.h"

namespace {

__device__ __forceinline__ int frame_of_view(const ExactArgs &A, int64_t view)
{
    int lo = 0, hi = A.nf;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (A.view_offset[mid] <= view) lo = mid;
        else hi = mid;
    }
    return lo;
}

// z[ray] = Lambda (y - A x) in FP64, every ray of every frame
__global__ __launch_bounds__(256) void k_exact_residual_sino(const ExactArgs A, const double *__restrict__ x,
                                                             const float *__restrict__ y,
                                                             const float *__restrict__ lam, double *__restrict__ z)
{
    const int64_t per_view = (int64_t)A.nu * A.nv;
    const int64_t n = A.n_views * per_view;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t view = i / per_view;
        const int rem = (int)(i - view * per_view);
        const int iu = rem / A.nv, iv = rem - iu * A.nv;
        const double w = (double)lam[i];
        double acc = 0.0;
        if (w != 0.0) {
            const double *xf = x + (int64_t)frame_of_view(A, view) * A.nvox;
            double S[3], d[3];
            ray_of(A, view, iu, iv, S, d);
            traverse(A, S, d, [&](int64_t vox, double len) { acc += len * xf[vox]; });
        }
        z[i] = w * ((double)y[i] - acc);
    }
}

// out += A^T z in FP64 (hardware FP64 atomic adds)
__global__ __launch_bounds__(256) void k_exact_back(const ExactArgs A, const double *__restrict__ z,
                                                    double *__restrict__ out)
{
    const int64_t per_view = (int64_t)A.nu * A.nv;
    const int64_t n = A.n_views * per_view;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double zi = z[i];
        if (zi == 0.0) continue;
        const int64_t view = i / per_view;
        const int rem = (int)(i - view * per_view);
        const int iu = rem / A.nv, iv = rem - iu * A.nv;
        double *of = out + (int64_t)frame_of_view(A, view) * A.nvox;
        double S[3], d[3];
        ray_of(A, view, iu, iv, S, d);
        traverse(A, S, d, [&](int64_t vox, double len) { atomicAdd(of + vox, len * zi); });
    }
}

ExactArgs exact_args(const msf_plan &P)
{
    ExactArgs A;
    A.nx = P.nx; A.ny = P.ny; A.nz = P.nz; A.nu = P.nu; A.nv = P.nv; A.nf = P.nf;
    A.du = P.du; A.dv = P.dv; A.rs = P.rs; A.rsd = P.rsd; A.offu = P.offu; A.offv = P.offv;
    A.cs = P.d_cs;
    A.view_offset = P.d_view_offset;
    A.n_views = P.n_views;
    A.nvox = P.nvox;
    return A;
}

unsigned ray_grid(int64_t n)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 20));
}

}  // namespace

// bp = A^T Lambda (y - A x) with FP64 lengths, sinogram and sums for an FP64
// volume x (bp zeroed first); the plan's sinograms sy, slam hold y and Lambda,
// and z64 is an FP64 sinogram of workspace.
hipError_t launch_exact_data_residual(msf_plan &P, const double *x, double *z64, hipStream_t s)
{
    const ExactArgs A = exact_args(P);
    hipError_t e = launch_fill_d(P.bp, P.nvox_total, s);
    if (e != hipSuccess || P.nmeas_total == 0) return e;
    hipLaunchKernelGGL(k_exact_residual_sino, dim3(ray_grid(P.nmeas_total)), dim3(256), 0, s, A, x, P.sy, P.slam,
                       z64);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_exact_back, dim3(ray_grid(P.nmeas_total)), dim3(256), 0, s, A, z64, P.bp);
    return hipGetLastError();
}
