// Learned warm start of the proximal-map solve: a 4-layer 3D CNN
// (3x3x3 kernels, channels 2 -> 16 -> 16 -> 16 -> 1, ReLU after the first
// three layers) predicting x0 = v + c_o f(v / c_v, g / c_g), where g is the
// data term's backprojected weighted residual at v in voxel units and c_v,
// c_g, c_o are fixed scales stored with the network.  The paper has no such network (its denoisers are 2.5D CNNs of
// a different kind); plain CG remains the fallback and the judge of the
// prediction.
//
// Every layer is an implicit GEMM on the matrix cores: channels-last BF16
// activations [N][Z][Y][X][16] (the 2-channel input and the 1-channel output
// are zero-padded to 16), and for each of the 27 taps one
// v_mfma_f32_16x16x16_bf16 multiplies 16 output voxels x 16 input channels by
// the tap's 16 x 16 weight block, accumulating in FP32.  The input gradient is
// the same kernel run with the spatially flipped, channel-transposed weights;
// the weight gradient is a split-K MFMA GEMM over voxels with a fixed-order
// reduction of the per-wave partial sums.  Master weights and Adam moments are
// FP32 (Adam: Kingma & Ba 2015).
#include "msf_internal.h"

#include <cmath>
#include <cstring>
#include <new>

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

constexpr int CH = 16;
constexpr int TAPS = 27;
constexpr int NPARAM = 15169;
constexpr int CIN[4] = {2, 16, 16, 16};
constexpr int COUT[4] = {16, 16, 16, 1};
constexpr int POFF[4] = {0, 880, 7808, 14736};   // offsets of W_l, b_l in the flat parameter vector
constexpr int WPACK = TAPS * CH * CH;              // packed bf16 weights per layer
constexpr int PART = TAPS * CH * CH + CH;          // weight-gradient partial per wave (+ bias)
constexpr int WG_BLOCKS = 512;                     // blocks of the weight-gradient kernel

enum Epi : int { EPI_RELU = 0, EPI_RESID = 1, EPI_MASK = 2 };

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct ConvArgs {
    const uint16_t *in;     // [N][Z][Y][X][16] bf16
    const uint16_t *w;      // [27][16 out][16 in] bf16
    const float *bias;      // [16] or nullptr
    int N, Z, Y, X;
    uint16_t *out_bf;       // EPI_RELU / EPI_MASK
    const uint16_t *mask;   // EPI_MASK: gradient passes where this activation is > 0
    float *out_f;           // EPI_RESID: x0 [N][Z][Y][X]
    const float *v;         // EPI_RESID
    float scale;            // EPI_RESID
};

template <int EPI>
__global__ __launch_bounds__(256) void k_conv(const ConvArgs A)
{
    __shared__ v4s wl[TAPS * CH * 4];   // [tap][out][k-group]: 4 input channels each
    const v4s *wsrc = reinterpret_cast<const v4s *>(A.w);
    for (int i = threadIdx.x; i < TAPS * CH * 4; i += blockDim.x) wl[i] = wsrc[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int nsx = (A.X + 15) / 16;
    const int64_t nseg = (int64_t)A.N * A.Z * A.Y * nsx;
    for (int64_t seg = (int64_t)blockIdx.x * 4 + wave; seg < nseg; seg += (int64_t)gridDim.x * 4) {
        int64_t t = seg;
        const int xs = (int)(t % nsx); t /= nsx;
        const int y = (int)(t % A.Y); t /= A.Y;
        const int z = (int)(t % A.Z);
        const int n = (int)(t / A.Z);
        const int x0 = xs * 16;
        v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int dz = 0; dz < 3; ++dz) {
            const int zz = z + dz - 1;
            const bool zok = zz >= 0 && zz < A.Z;
            for (int dy = 0; dy < 3; ++dy) {
                const int yy = y + dy - 1;
                const bool yok = zok && yy >= 0 && yy < A.Y;
                const int64_t row = (((int64_t)n * A.Z + zz) * A.Y + yy) * A.X;
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int xx = x0 + r + dx - 1;
                    v4s a = {0, 0, 0, 0};
                    if (yok && xx >= 0 && xx < A.X) a = *reinterpret_cast<const v4s *>(A.in + (row + xx) * CH + 4 * g);
                    const v4s b = wl[((dz * 3 + dy) * 3 + dx) * (CH * 4) + r * 4 + g];
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
                }
            }
        }
        // lane holds output voxel x0 + 4g + j, channel r
        const float bias = A.bias ? A.bias[r] : 0.0f;
        const int64_t vrow = (((int64_t)n * A.Z + z) * A.Y + y) * A.X;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int xv = x0 + 4 * g + j;
            if (xv >= A.X) continue;
            const int64_t vox = vrow + xv;
            const float val = acc[j] + bias;
            if (EPI == EPI_RELU) {
                A.out_bf[vox * CH + r] = f2bf(fmaxf(val, 0.0f));
            } else if (EPI == EPI_MASK) {
                A.out_bf[vox * CH + r] = bf2f(A.mask[vox * CH + r]) > 0.0f ? f2bf(val) : (uint16_t)0;
            } else {
                if (r == 0) A.out_f[vox] = A.v[vox] + A.scale * val;
            }
        }
    }
}

struct WgradArgs {
    const uint16_t *g;      // [N][Z][Y][X][16] gradient at the layer output (bf16)
    const uint16_t *h;      // [N][Z][Y][X][16] layer input (bf16)
    int N, Z, Y, X;
    float *part;            // [n_waves][PART]
};

// dW[tap][o][i] = sum_p g[p][o] h[p + tap - 1][i]: M = o, N = i, K = voxels.
__global__ __launch_bounds__(256) void k_wgrad(const WgradArgs A)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int nsx = (A.X + 15) / 16;
    const int64_t nseg = (int64_t)A.N * A.Z * A.Y * nsx;
    v4f acc[TAPS];
#pragma unroll
    for (int k = 0; k < TAPS; ++k) acc[k] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    for (int64_t seg = (int64_t)blockIdx.x * 4 + wave; seg < nseg; seg += (int64_t)gridDim.x * 4) {
        int64_t t = seg;
        const int xs = (int)(t % nsx); t /= nsx;
        const int y = (int)(t % A.Y); t /= A.Y;
        const int z = (int)(t % A.Z);
        const int n = (int)(t / A.Z);
        const int x0 = xs * 16;
        const int64_t vrow = (((int64_t)n * A.Z + z) * A.Y + y) * A.X;
        v4s ga;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int xv = x0 + 4 * g + j;
            const uint16_t gv = xv < A.X ? A.g[(vrow + xv) * CH + r] : (uint16_t)0;
            ga[j] = (short)gv;
            bsum += bf2f(gv);
        }
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            const int zz = z + dz - 1;
            const bool zok = zz >= 0 && zz < A.Z;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const int yy = y + dy - 1;
                const bool yok = zok && yy >= 0 && yy < A.Y;
                const int64_t row = (((int64_t)n * A.Z + zz) * A.Y + yy) * A.X;
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    v4s hb;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int xv = x0 + 4 * g + j;
                        const int xx = xv + dx - 1;
                        hb[j] = (short)((yok && xv < A.X && xx >= 0 && xx < A.X) ? A.h[(row + xx) * CH + r] : (uint16_t)0);
                    }
                    const int tap = (dz * 3 + dy) * 3 + dx;
                    acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ga, hb, acc[tap], 0, 0, 0);
                }
            }
        }
    }
    float *out = A.part + ((int64_t)blockIdx.x * 4 + wave) * PART;
#pragma unroll
    for (int k = 0; k < TAPS; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) out[k * CH * CH + (4 * g + j) * CH + r] = acc[k][j];
    // bias gradient of output channel r: the four lanes r, r+16, r+32, r+48
    bsum += __shfl_xor(bsum, 16, 64);
    bsum += __shfl_xor(bsum, 32, 64);
    if (g == 0) out[TAPS * CH * CH + r] = bsum;
}

// grad_flat[layer] <- sum of the per-wave partials (fixed order), real channels only
__global__ void k_wgrad_reduce(const float *__restrict__ part, int nwaves, int layer, float *__restrict__ grad)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= PART) return;
    float s = 0.0f;
    for (int w = 0; w < nwaves; ++w) s += part[(int64_t)w * PART + e];
    const int cin = CIN[layer], cout = COUT[layer];
    if (e < TAPS * CH * CH) {
        const int tap = e / (CH * CH), o = (e / CH) % CH, i = e % CH;
        if (o < cout && i < cin) grad[POFF[layer] + (o * cin + i) * TAPS + tap] = s;
    } else {
        const int o = e - TAPS * CH * CH;
        if (o < cout) grad[POFF[layer] + cout * cin * TAPS + o] = s;
    }
}

// bf16 weights for the forward ([tap][out][in]) and the input gradient
// (flipped taps, in/out swapped), FP32 biases padded to 16
__global__ void k_pack(const float *__restrict__ master, uint16_t *__restrict__ wf, uint16_t *__restrict__ wd,
                       float *__restrict__ bias)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 4 * WPACK) return;
    const int layer = e / WPACK, k = e % WPACK;
    const int tap = k / (CH * CH), o = (k / CH) % CH, i = k % CH;
    const int cin = CIN[layer], cout = COUT[layer];
    const float *W = master + POFF[layer];
    wf[e] = (o < cout && i < cin) ? f2bf(W[(o * cin + i) * TAPS + tap]) : (uint16_t)0;
    // input gradient: out channel o' = forward input i', in channel i' = forward output o'
    const int ftap = TAPS - 1 - tap;
    wd[e] = (i < cout && o < cin) ? f2bf(W[(i * cin + o) * TAPS + ftap]) : (uint16_t)0;
    if (k < CH) bias[layer * CH + k] = k < cout ? master[POFF[layer] + cout * cin * TAPS + k] : 0.0f;
}

// input channels: bf16(v / c_v), bf16(g / c_g), zeros
__global__ void k_pack_input(const float *__restrict__ v, const float *__restrict__ gin, int64_t n, float inv_cv,
                             float inv_cg, uint16_t *__restrict__ h0)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * CH; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t vox = e / CH;
        const int c = (int)(e % CH);
        h0[e] = c == 0 ? f2bf(v[vox] * inv_cv) : (c == 1 ? f2bf(gin[vox] * inv_cg) : (uint16_t)0);
    }
}

// loss partials (FP64) and the output gradient bf16(2 (x0 - t) / n * c) in channel 0
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ pred, const float *__restrict__ tgt, int64_t n,
                                             float gscale, uint16_t *__restrict__ g4, double *__restrict__ part)
{
    double s = 0.0;
    for (int64_t vox = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; vox < n; vox += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)pred[vox] - (double)tgt[vox];
        s += d * d;
        g4[vox * CH] = f2bf((float)(2.0 * d / (double)n) * gscale);
        for (int c = 1; c < CH; ++c) g4[vox * CH + c] = 0;
    }
    __shared__ double red[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ grad, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gv = grad[e];
    const float mm = b1 * m[e] + (1.0f - b1) * gv;
    const float vv = b2 * v[e] + (1.0f - b2) * gv * gv;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void k_count_nonfinite(const float *__restrict__ a, int64_t n, int32_t *__restrict__ flag)
{
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad += !isfinite(a[i]);
    if (bad) atomicAdd(flag, bad);
}

unsigned grid_of(int64_t work, int per_block)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

struct msf_cnn {
    float cv = 1.0f, cg = 1.0f, co = 1.0f;   // input / feature / output scales
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t *wf = nullptr, *wd = nullptr;
    float *bias = nullptr;
    // activation workspace sized for cap voxels
    int64_t cap = 0;
    uint16_t *h[4] = {nullptr, nullptr, nullptr, nullptr};
    uint16_t *ga = nullptr, *gb = nullptr;
    float *pred = nullptr;
    float *part = nullptr;
    double *lpart = nullptr;
    double *hlpart = nullptr;
    int32_t *flag = nullptr;
    int64_t step = 0;
    // public-layout feature / prediction volumes used inside the solver
    float *io = nullptr;
    int64_t io_cap = 0;
};

namespace {

template <class T>
hipError_t cnn_alloc(T **p, size_t n)
{
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

void cnn_free_ws(msf_cnn *C)
{
    for (auto &q : C->h)
        if (q) (void)hipFree(q), q = nullptr;
    void *ps[] = {C->ga, C->gb, C->pred};
    for (void *q : ps)
        if (q) (void)hipFree(q);
    C->ga = C->gb = nullptr;
    C->pred = nullptr;
    C->cap = 0;
}

hipError_t cnn_reserve(msf_cnn *C, int64_t nvox)
{
    if (nvox <= C->cap) return hipSuccess;
    cnn_free_ws(C);
    hipError_t e;
    for (auto &q : C->h)
        if ((e = cnn_alloc(&q, (size_t)nvox * CH)) != hipSuccess) return e;
    if ((e = cnn_alloc(&C->ga, (size_t)nvox * CH)) != hipSuccess) return e;
    if ((e = cnn_alloc(&C->gb, (size_t)nvox * CH)) != hipSuccess) return e;
    if ((e = cnn_alloc(&C->pred, (size_t)nvox)) != hipSuccess) return e;
    C->cap = nvox;
    return hipSuccess;
}

hipError_t launch_conv(int epi, const uint16_t *in, const uint16_t *w, const float *bias, int N, int Z, int Y, int X,
                       uint16_t *out_bf, const uint16_t *mask, float *out_f, const float *v, float scale, hipStream_t s)
{
    ConvArgs A{in, w, bias, N, Z, Y, X, out_bf, mask, out_f, v, scale};
    const int64_t nseg = (int64_t)N * Z * Y * ((X + 15) / 16);
    const dim3 grid(grid_of(nseg, 4)), block(256);
    switch (epi) {
    case EPI_RELU: hipLaunchKernelGGL(k_conv<EPI_RELU>, grid, block, 0, s, A); break;
    case EPI_MASK: hipLaunchKernelGGL(k_conv<EPI_MASK>, grid, block, 0, s, A); break;
    default: hipLaunchKernelGGL(k_conv<EPI_RESID>, grid, block, 0, s, A); break;
    }
    return hipGetLastError();
}

hipError_t cnn_forward(msf_cnn *C, const float *v, const float *gin, int N, int Z, int Y, int X, float *x0,
                       hipStream_t s)
{
    const int64_t n = (int64_t)N * Z * Y * X;
    hipError_t e;
    hipLaunchKernelGGL(k_pack_input, dim3(grid_of(n * CH, 256)), dim3(256), 0, s, v, gin, n, 1.0f / C->cv,
                       1.0f / C->cg, C->h[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int l = 0; l < 3; ++l)
        if ((e = launch_conv(EPI_RELU, C->h[l], C->wf + l * WPACK, C->bias + l * CH, N, Z, Y, X, C->h[l + 1],
                             nullptr, nullptr, nullptr, 0.0f, s)) != hipSuccess)
            return e;
    return launch_conv(EPI_RESID, C->h[3], C->wf + 3 * WPACK, C->bias + 3 * CH, N, Z, Y, X, nullptr, nullptr, x0, v,
                       C->co, s);
}

hipError_t cnn_pack(msf_cnn *C, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack, dim3((4 * WPACK + 255) / 256), dim3(256), 0, s, C->master, C->wf, C->wd, C->bias);
    return hipGetLastError();
}

#define CHK(expr)                                            \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

}  // namespace

hipError_t cnn_io_buffers(msf_cnn *C, int64_t n, float **g, float **x)
{
    if (n > C->io_cap) {
        if (C->io) (void)hipFree(C->io);
        C->io = nullptr;
        C->io_cap = 0;
        hipError_t e = cnn_alloc(&C->io, (size_t)(2 * n));
        if (e != hipSuccess) return e;
        C->io_cap = n;
    }
    *g = C->io;
    *x = C->io + n;
    return hipSuccess;
}

hipError_t cnn_infer_internal(msf_cnn *C, const float *v, const float *g, int N, int Z, int Y, int X, float *x0,
                              hipStream_t s)
{
    // volumes are independent: evaluate them in chunks of at most 2^26 voxels
    // (activations take 32 bytes per voxel and layer)
    const int64_t per = (int64_t)Z * Y * X;
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(N, ((int64_t)1 << 26) / per));
    hipError_t e = cnn_reserve(C, (int64_t)chunk * per);
    if (e != hipSuccess) return e;
    for (int f0 = 0; f0 < N; f0 += chunk) {
        const int nf = std::min(chunk, N - f0);
        e = cnn_forward(C, v + f0 * per, g + f0 * per, nf, Z, Y, X, x0 + f0 * per, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

extern "C" {

msf_status msf_cnn_create(const float *params, int64_t n_params, const float *scales, msf_cnn **out)
{
    set_error("");
    if (!params || !out || !scales || n_params != NPARAM) {
        set_error("msf_cnn_create: need 15169 parameters and 3 scales");
        return MSF_EINVAL;
    }
    for (int k = 0; k < 3; ++k)
        if (!(std::isfinite(scales[k]) && scales[k] > 0.0f)) {
            set_error("msf_cnn_create: scales must be positive and finite");
            return MSF_EINVAL;
        }
    for (int64_t i = 0; i < n_params; ++i)
        if (!std::isfinite(params[i])) { set_error("msf_cnn_create: non-finite parameter"); return MSF_EINVAL; }
    msf_cnn *C = new (std::nothrow) msf_cnn();
    if (!C) { set_error("host allocation failed"); return MSF_ENOMEM; }
    C->cv = scales[0];
    C->cg = scales[1];
    C->co = scales[2];
    hipError_t e = hipSuccess;
    auto fail = [&](hipError_t err) {
        msf_cnn_destroy(C);
        return hip_fail(err, "msf_cnn_create");
    };
    if ((e = cnn_alloc(&C->master, NPARAM)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->m, NPARAM)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->v, NPARAM)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->grad, NPARAM)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->wf, 4 * WPACK)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->wd, 4 * WPACK)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->bias, 4 * CH)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->part, (size_t)WG_BLOCKS * 4 * PART)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->lpart, 65536)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->flag, 4)) != hipSuccess) return fail(e);
    if ((e = hipHostMalloc((void **)&C->hlpart, 65536 * sizeof(double), hipHostMallocDefault)) != hipSuccess) return fail(e);
    if ((e = hipMemcpy(C->master, params, NPARAM * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
    if ((e = hipMemset(C->m, 0, NPARAM * sizeof(float))) != hipSuccess) return fail(e);
    if ((e = hipMemset(C->v, 0, NPARAM * sizeof(float))) != hipSuccess) return fail(e);
    if ((e = cnn_pack(C, nullptr)) != hipSuccess) return fail(e);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(e);
    *out = C;
    return MSF_OK;
}

void msf_cnn_destroy(msf_cnn *C)
{
    if (!C) return;
    (void)hipDeviceSynchronize();
    cnn_free_ws(C);
    void *ps[] = {C->master, C->m, C->v, C->grad, C->wf, C->wd, C->bias, C->part, C->lpart, C->flag, C->io};
    for (void *q : ps)
        if (q) (void)hipFree(q);
    if (C->hlpart) (void)hipHostFree(C->hlpart);
    delete C;
}

msf_status msf_cnn_get_params(const msf_cnn *C, float *params)
{
    if (!C || !params) { set_error("null argument"); return MSF_EINVAL; }
    CHK(hipMemcpy(params, C->master, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    return MSF_OK;
}

msf_status msf_cnn_infer(msf_cnn *C, const float *v, const float *g, int32_t n, int32_t nz, int32_t ny, int32_t nx,
                         float *x0, void *stream)
{
    set_error("");
    if (!C || !v || !g || !x0 || n <= 0 || nz <= 0 || ny <= 0 || nx <= 0) { set_error("invalid argument"); return MSF_EINVAL; }
    CHK(cnn_infer_internal(C, v, g, n, nz, ny, nx, x0, (hipStream_t)stream));
    return MSF_OK;
}

msf_status msf_cnn_train_step(msf_cnn *C, const float *v, const float *g, const float *target, int32_t n, int32_t nz,
                              int32_t ny, int32_t nx, double lr, int32_t apply, double *loss_out, float *grad_out,
                              void *stream)
{
    set_error("");
    if (!C || !v || !g || !target || n <= 0 || nz <= 0 || ny <= 0 || nx <= 0 || !(lr >= 0.0)) {
        set_error("invalid argument");
        return MSF_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t nvox = (int64_t)n * nz * ny * nx;
    CHK(cnn_reserve(C, nvox));
    CHK(cnn_forward(C, v, g, n, nz, ny, nx, C->pred, s));
    const unsigned lb = grid_of(nvox, 256);
    hipLaunchKernelGGL(k_mse, dim3(lb), dim3(256), 0, s, C->pred, target, nvox, C->co, C->ga, C->lpart);
    CHK(hipGetLastError());
    // backward: g_l is the gradient at layer l's output (bf16, ReLU mask applied)
    uint16_t *gcur = C->ga, *gnext = C->gb;
    for (int l = 3; l >= 0; --l) {
        WgradArgs W{gcur, C->h[l], n, nz, ny, nx, C->part};
        hipLaunchKernelGGL(k_wgrad, dim3(WG_BLOCKS), dim3(256), 0, s, W);
        CHK(hipGetLastError());
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((PART + 255) / 256), dim3(256), 0, s, C->part, WG_BLOCKS * 4, l,
                           C->grad);
        CHK(hipGetLastError());
        if (l > 0) {
            CHK(launch_conv(EPI_MASK, gcur, C->wd + l * WPACK, nullptr, n, nz, ny, nx, gnext, C->h[l], nullptr,
                            nullptr, 0.0f, s));
            std::swap(gcur, gnext);
        }
    }
    CHK(hipMemcpyAsync(C->hlpart, C->lpart, lb * sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad_out) CHK(hipMemcpyAsync(grad_out, C->grad, NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
    if (apply) {
        C->step++;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - std::pow(b1, (float)C->step), c2 = 1.0f - std::pow(b2, (float)C->step);
        hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, C->master, C->m, C->v, C->grad,
                           NPARAM, (float)lr, b1, b2, 1e-8f, c1, c2);
        CHK(hipGetLastError());
        CHK(cnn_pack(C, s));
    }
    CHK(hipStreamSynchronize(s));
    double loss = 0.0;
    for (unsigned b = 0; b < lb; ++b) loss += C->hlpart[b];
    if (loss_out) *loss_out = loss / (double)nvox;
    return MSF_OK;
}

}  // extern "C"
