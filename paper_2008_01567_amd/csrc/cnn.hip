// Two networks share these kernels.
//
// The learned warm start of the proximal-map solve: a 4-layer 3D CNN
// (3x3x3 kernels, channels 2 -> 16 -> 16 -> 16 -> 1, ReLU after the first
// three layers) predicting x0 = v + c_o f(v / c_v, g / c_g), where g is the
// data term's backprojected weighted residual at v in voxel units and c_v,
// c_g, c_o are fixed scales stored with the network.  The paper has no such
// network; plain CG remains the fallback and decides whether the prediction is kept.
//
// The 2.5D denoiser of the multi-slice fusion prior agents (paper Sec. IV):
// the same four layers as a 2D network (3x3 kernels, channels 5 -> 16 -> 16
// -> 16 -> 1) whose five input channels are one 2D slice at five adjacent
// time points t-2 .. t+2 and whose output is the denoised centre slice,
// x = s_t + c_o f(s_{t-2..t+2} / c_in).  Images are 2D (depth 1); the depth
// taps of the 3D kernels are skipped.
//
// Every layer is an implicit GEMM on the matrix cores: channels-last BF16
// activations [N][Z][Y][X][16] (the 2- or 5-channel input and the 1-channel
// output are zero-padded to 16), and each v_mfma_f32_16x16x32_bf16 multiplies
// 16 output channels by 16 voxels over K = 32 (tap, input channel) pairs,
// accumulating in FP32: two taps of 16 channels each, or, where only the
// first 8 channels can be nonzero (the denoiser's first layer), four taps of
// 8.  Lane (r, g) of the wave supplies the 8 K values 8g .. 8g + 7 for output
// channel r (weights) and voxel r (activations), the latter with one 16-byte
// LDS read.  Input rows are staged in
// LDS by workgroup tiles (2D images: row tiles; 3D volumes: row tiles sliding
// along z with a three-slice ring), zero outside the volume.  The input gradient is
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
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));

namespace {

constexpr int CH = 16;
constexpr int TAPS = 27;
constexpr int COUT[4] = {16, 16, 16, 1};
constexpr int WPACK = TAPS * CH * CH;              // packed bf16 weights per layer
constexpr int PART = TAPS * CH * CH + CH;          // weight-gradient partial per wave (+ bias)
constexpr int WG_BLOCKS = 512;                     // blocks of the weight-gradient kernel

enum Epi : int { EPI_RELU = 0, EPI_RESID = 1, EPI_MASK = 2 };

// Parameter layout of a network: per layer W[out][in][taps] then b[out],
// with taps = 27 (3x3x3) or 9 (3x3, the depth-centre taps of the kernels).
struct NetShape {
    int cin0;             // input channels of the first layer (2 or 5)
    int ptaps;            // 27 or 9
    int poff[4];          // offsets of W_l, b_l in the flat parameter vector
    int nparam;
};

__host__ __device__ inline int net_cin(const NetShape &S, int layer) { return layer == 0 ? S.cin0 : CH; }

// parameter tap of kernel tap (dz, dy, dx), or -1 for a depth tap of a 2D network
__host__ __device__ inline int net_ptap(const NetShape &S, int tap)
{
    if (S.ptaps == TAPS) return tap;
    return tap / 9 == 1 ? tap - 9 : -1;
}

NetShape make_shape(int cin0, int ptaps)
{
    NetShape S{};
    S.cin0 = cin0;
    S.ptaps = ptaps;
    int o = 0;
    for (int l = 0; l < 4; ++l) {
        S.poff[l] = o;
        o += COUT[l] * (net_cin(S, l) * ptaps + 1);
    }
    S.nparam = o;
    return S;
}

// FP32 -> BF16, round to nearest even (the hardware conversion of gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// two values, packed low | high << 16, in one conversion
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){lo, hi}, bf16x2_t));
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Sources of the input channels of images [n0, n0 + n / per):
//   IN_WARM:  channel 0 = a / c_v, channel 1 = g / c_g (volumes [img][per]);
//   IN_STACK: channel c = a[img][c][per] / c_in, c < 5;
//   IN_SEQ:   a is a sequence [T][S][per] of S images per time point; image
//             t S + s has channel c = the same image at time clamp(t + c - 2)
//             / c_in, c < 5 (time points t-2 .. t+2, repeated at the ends).
enum InMode : int { IN_WARM = 0, IN_STACK = 1, IN_SEQ = 2 };

struct PackIn {
    int mode;
    const float *a, *g;
    int64_t n0;           // first image (IN_SEQ)
    int T, S;             // IN_SEQ
    float inv0, inv1;
};

__device__ __forceinline__ float pack_src(const PackIn &P, int64_t img, int64_t loc, int c, int64_t per)
{
    if (P.mode == IN_WARM) return c == 0 ? P.a[img * per + loc] : P.g[img * per + loc];
    if (P.mode == IN_STACK) return P.a[(img * 5 + c) * per + loc];
    const int64_t gi = P.n0 + img;
    const int t = (int)(gi / P.S), si = (int)(gi - (int64_t)t * P.S);
    const int tt = min(max(t + c - 2, 0), P.T - 1);
    return P.a[((int64_t)tt * P.S + si) * per + loc];
}

struct ConvArgs {
    const uint16_t *in;     // [N][Z][Y][X][16] bf16
    const uint16_t *w;      // [27][16 out][16 in] bf16
    const float *bias;      // [16] or nullptr
    int N, Z, Y, X;
    uint16_t *out_bf;       // EPI_RELU / EPI_MASK
    const uint16_t *mask;   // EPI_MASK: gradient passes where this activation is > 0
    float *out_f;           // EPI_RESID: x0 [N][Z][Y][X]
    const float *v;         // EPI_RESID: residual base of image n at v + n * v_stride + v_off
    int64_t v_stride, v_off;
    float scale;            // EPI_RESID
    PackIn pin;             // k_conv2d<.., true>: the FP32 sources of the first layer's input channels
};

// The MFMAs take the weights as the A operand and the activations as B, so
// lane (r, g) ends with output channels 4g .. 4g + 3 of voxel r of its
// segment: one 8-byte store per lane, 512 contiguous bytes per wave.
template <int EPI>
__device__ __forceinline__ void conv_store(const ConvArgs &A, const v4f &acc, const float4 &b, int64_t vox,
                                           int64_t vres, int g)
{
    const float o[4] = {acc[0] + b.x, acc[1] + b.y, acc[2] + b.z, acc[3] + b.w};
    if (EPI == EPI_RELU) {
        uint2 w;
        w.x = f2bf2(fmaxf(o[0], 0.0f), fmaxf(o[1], 0.0f));
        w.y = f2bf2(fmaxf(o[2], 0.0f), fmaxf(o[3], 0.0f));
        *reinterpret_cast<uint2 *>(A.out_bf + vox * CH + 4 * g) = w;
    } else if (EPI == EPI_MASK) {
        const uint2 m = *reinterpret_cast<const uint2 *>(A.mask + vox * CH + 4 * g);
        const uint16_t mk[4] = {(uint16_t)(m.x & 0xFFFFu), (uint16_t)(m.x >> 16), (uint16_t)(m.y & 0xFFFFu),
                                (uint16_t)(m.y >> 16)};
        uint16_t h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) h[j] = bf2f(mk[j]) > 0.0f ? f2bf(o[j]) : (uint16_t)0;
        *reinterpret_cast<uint2 *>(A.out_bf + vox * CH + 4 * g) =
            make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
    } else {
        if (g == 0) A.out_f[vox] = A.v[vres] + A.scale * o[0];
    }
}

__device__ __forceinline__ float4 conv_bias(const ConvArgs &A, int g)
{
    return A.bias ? *reinterpret_cast<const float4 *>(A.bias + 4 * g) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Depth-1 images (the 2.5D denoiser): a workgroup owns a tile of TY rows x
// 64 voxels of one image and stages its input rows plus a one-voxel halo in
// LDS with 16-byte coalesced loads, so each input voxel is read from memory
// about (TY + 2) / TY times instead of nine; wave w computes the 16-voxel
// segment 16w .. 16w + 15 of every row of the tile from LDS.  The next
// tile's rows are loaded into registers while the current one is multiplied.
constexpr int TY = 8, TXW = 64, TROW = TXW + 2;
constexpr int TILE_U4 = (TY + 2) * TROW * 2;          // 16-byte chunks in the staged rows
constexpr int TILE_LD = (TILE_U4 + 255) / 256;        // per thread

// 8 BF16 values at a 16-byte aligned v4s pair (weights or staged channels)
__device__ __forceinline__ v8bf ld8(const v4s *p) { return __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4 *>(p)); }

// The K slots of one 16x16x32 MFMA over a 3x3 window: TPM taps of 32 / TPM
// channels each (TPM = 2: all 16 channels; TPM = 4: channels 0 .. 7).  Lane
// group g takes tap TPM m + g / (4 / TPM) of MFMA m and channel block
// c = (g % (4 / TPM)) * 8; taps past the window get zero weights (and read
// tap 0's voxel, a finite value).  For tap (dy, dx) the staged voxel of output
// column r is at (dy * TROW + dx + r) * 4 + c / 4 in v4s units.
template <int TPM>
struct Window {
    static constexpr int M = (9 + TPM - 1) / TPM;   // MFMAs per output row
    v8bf w[M];
    int off[M];
    __device__ __forceinline__ void load(const v4s *wl, int tap0, int r, int g)
    {
        constexpr int per = 4 / TPM;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int tap = TPM * m + g / per, c4 = (g % per) * 2;
            const bool real = tap < 9;
            const v8bf zero = {};
            w[m] = real ? ld8(wl + (tap0 + (real ? tap : 0)) * (CH * 4) + r * 4 + c4) : zero;
            off[m] = real ? ((tap / 3) * TROW + tap % 3) * 4 + c4 : c4;
        }
    }
    // acc += this window applied at staged position base (v4s units, column r included)
    __device__ __forceinline__ void apply(const v4s *tl, int base, v4f &acc) const
    {
#pragma unroll
        for (int m = 0; m < M; ++m)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[m], ld8(tl + base + off[m]), acc, 0, 0, 0);
    }
};

struct TilePos {
    int n, y0, x0;
};

__device__ __forceinline__ TilePos tile_pos(int64_t t, int ntx, int nty)
{
    TilePos p;
    p.x0 = (int)(t % ntx) * TXW;
    t /= ntx;
    p.y0 = (int)(t % nty) * TY;
    p.n = (int)(t / nty);
    return p;
}

__device__ __forceinline__ void tile_fetch(const ConvArgs &A, const TilePos &p, uint4 (&reg)[TILE_LD])
{
    const uint4 *src = reinterpret_cast<const uint4 *>(A.in);
#pragma unroll
    for (int k = 0; k < TILE_LD; ++k) {
        const int idx = threadIdx.x + 256 * k;
        const int row = idx / (2 * TROW), rem = idx - row * (2 * TROW);
        const int gy = p.y0 - 1 + row, gx = p.x0 - 1 + (rem >> 1);
        const bool ok = idx < TILE_U4 && gy >= 0 && gy < A.Y && gx >= 0 && gx < A.X;
        reg[k] = ok ? src[(((int64_t)p.n * A.Y + gy) * A.X + gx) * 2 + (rem & 1)] : make_uint4(0, 0, 0, 0);
    }
}

// First layer straight from the FP32 sources: each thread stages whole voxels
// (its input channels scaled and rounded to BF16 as the input pack does).
constexpr int TILE_VOX = (TY + 2) * TROW;
constexpr int TILE_VLD = (TILE_VOX + 255) / 256;      // voxels per thread

__device__ __forceinline__ void tile_fetch_f32(const ConvArgs &A, const TilePos &p, float (&reg)[TILE_VLD][5])
{
    // the tile's image is one image: its channel planes and scales are uniform
    const PackIn &P = A.pin;
    const int64_t per = (int64_t)A.Y * A.X;
    const int cin = P.mode == IN_WARM ? 2 : 5;
    const float *ch[5];
    float sc[5];
    if (P.mode == IN_SEQ) {
        const int64_t gi = P.n0 + p.n;
        const int t = (int)(gi / P.S), si = (int)(gi - (int64_t)t * P.S);
#pragma unroll
        for (int c = 0; c < 5; ++c) ch[c] = P.a + ((int64_t)min(max(t + c - 2, 0), P.T - 1) * P.S + si) * per;
    } else if (P.mode == IN_STACK) {
#pragma unroll
        for (int c = 0; c < 5; ++c) ch[c] = P.a + ((int64_t)p.n * 5 + c) * per;
    } else {
        ch[0] = P.a + (int64_t)p.n * per;
        ch[1] = P.g + (int64_t)p.n * per;
        ch[2] = ch[3] = ch[4] = ch[0];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) sc[c] = (P.mode == IN_WARM && c == 1) ? P.inv1 : P.inv0;
#pragma unroll
    for (int k = 0; k < TILE_VLD; ++k) {
        const int vi = threadIdx.x + 256 * k;
        const int row = vi / TROW, col = vi - row * TROW;
        const int gy = p.y0 - 1 + row, gx = p.x0 - 1 + col;
        const bool ok = vi < TILE_VOX && gy >= 0 && gy < A.Y && gx >= 0 && gx < A.X;
        const int64_t loc = (int64_t)gy * A.X + gx;
#pragma unroll
        for (int c = 0; c < 5; ++c) reg[k][c] = (ok && c < cin) ? ch[c][loc] * sc[c] : 0.0f;
    }
}

__device__ __forceinline__ void tile_store_f32(uint4 *tile, const float (&reg)[TILE_VLD][5])
{
#pragma unroll
    for (int k = 0; k < TILE_VLD; ++k) {
        const int vi = threadIdx.x + 256 * k;
        if (vi >= TILE_VOX) continue;
        // f2bf(0) = 0, so the channels past the network's inputs stay zero
        tile[2 * vi] = make_uint4(f2bf2(reg[k][0], reg[k][1]), f2bf2(reg[k][2], reg[k][3]), f2bf2(reg[k][4], 0.0f), 0u);
        tile[2 * vi + 1] = make_uint4(0u, 0u, 0u, 0u);
    }
}

template <int EPI, bool F32IN>
__global__ __launch_bounds__(256) void k_conv2d(const ConvArgs A)
{
    __shared__ v4s wl[9 * CH * 4];
    __shared__ uint4 tile[TILE_U4];
    const v4s *wsrc = reinterpret_cast<const v4s *>(A.w) + 9 * CH * 4;     // the depth-centre taps
    for (int i = threadIdx.x; i < 9 * CH * 4; i += blockDim.x) wl[i] = wsrc[i];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int ntx = (A.X + TXW - 1) / TXW, nty = (A.Y + TY - 1) / TY;
    const int64_t ntile = (int64_t)A.N * nty * ntx;
    const float4 bias = conv_bias(A, g);
    int64_t t = blockIdx.x;
    if (t >= ntile) return;                  // the whole workgroup
    TilePos p = tile_pos(t, ntx, nty);
    __syncthreads();                         // the weights are staged
    // this lane's weight blocks, in registers; the first layer's inputs fill channels 0 .. 4 only
    Window<F32IN ? 4 : 2> win;
    win.load(wl, 0, r, g);
    uint4 reg[F32IN ? 1 : TILE_LD];
    float regf[F32IN ? TILE_VLD : 1][5];
    if constexpr (F32IN) tile_fetch_f32(A, p, regf);
    else tile_fetch(A, p, reg);
    const v4s *tl = reinterpret_cast<const v4s *>(tile);
    for (; t < ntile; t += gridDim.x) {
        __syncthreads();                     // the previous tile's reads are done
        if constexpr (F32IN) {
            tile_store_f32(tile, regf);
        } else {
#pragma unroll
            for (int k = 0; k < TILE_LD; ++k) {
                const int idx = threadIdx.x + 256 * k;
                if (idx < TILE_U4) tile[idx] = reg[k];
            }
        }
        __syncthreads();
        const TilePos pc = p;
        const int64_t tn = t + gridDim.x;
        if (tn < ntile) {
            p = tile_pos(tn, ntx, nty);
            if constexpr (F32IN) tile_fetch_f32(A, p, regf);
            else tile_fetch(A, p, reg);
        }
        const int xs = pc.x0 + 16 * wave;    // this wave's segment
        if (xs >= A.X) continue;             // wave-uniform; no barrier until the next tile
        // the residual output adds the tile's base values, loaded before the MFMAs (lanes g = 0 store)
        float vb[EPI == EPI_RESID ? TY : 1];
        if constexpr (EPI == EPI_RESID) {
#pragma unroll
            for (int ry = 0; ry < TY; ++ry) {
                const int y = pc.y0 + ry, xv = xs + r;
                vb[ry] = (g == 0 && y < A.Y && xv < A.X)
                             ? A.v[(int64_t)pc.n * A.v_stride + A.v_off + (int64_t)y * A.X + xv]
                             : 0.0f;
            }
        }
        for (int ry = 0; ry < TY && pc.y0 + ry < A.Y; ++ry) {
            v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
            // staged voxels (row ry + dy, column 16 wave + r + dx)
            win.apply(tl, (ry * TROW + 16 * wave + r) * 4, acc);
            const int y = pc.y0 + ry, xv = xs + r;
            const int64_t vox = ((int64_t)pc.n * A.Y + y) * A.X + xv;
            if constexpr (EPI == EPI_RESID) {
                if (xv < A.X && g == 0) A.out_f[vox] = vb[ry] + A.scale * (acc[0] + bias.x);
            } else {
                if (xv < A.X) conv_store<EPI>(A, acc, bias, vox, 0, g);
            }
        }
    }
}

// First layer of the 2.5D denoiser on a plane sequence [T][S][H][W] (IN_SEQ):
// a workgroup owns one (slice s, 8-row, 64-voxel) tile and walks along the
// time points [t0, t1) of the chunk.  Each thread keeps, for its staged
// voxels of the tile (halo included), the BF16 values of the frames
// clamp(t - 2) .. clamp(t + 2) (scaled as the input pack does) in registers,
// two to a dword, so each frame is read from memory once per tile.  Per time
// point it writes them as channels 0 .. 4 of the staged tile, in the layout
// of the other layers (16 channels per voxel, 5 .. 15 zero), and the MFMAs
// read one 8-byte operand per tap.  Frame t + 3 is loaded into registers while
// time point t is multiplied.
constexpr int RING_VOX = (TY + 2) * TROW;
constexpr int RING_LD = (RING_VOX + 255) / 256;

__device__ __forceinline__ void frame_fetch(const ConvArgs &A, int f, int s, int y0, int x0, float (&reg)[RING_LD])
{
    const PackIn &P = A.pin;
    const int64_t per = (int64_t)A.Y * A.X;
    const float *src = P.a + ((int64_t)f * P.S + s) * per;
#pragma unroll
    for (int k = 0; k < RING_LD; ++k) {
        const int vi = threadIdx.x + 256 * k;
        const int row = vi / TROW, col = vi - row * TROW;
        const int gy = y0 - 1 + row, gx = x0 - 1 + col;
        const bool ok = vi < RING_VOX && f >= 0 && f < P.T && gy >= 0 && gy < A.Y && gx >= 0 && gx < A.X;
        reg[k] = ok ? src[(int64_t)gy * A.X + gx] * P.inv0 : 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_conv2d_first_seq(const ConvArgs A, int t0, int t1)
{
    __shared__ v4s wl[9 * CH * 4];
    __shared__ uint4 tile[2 * RING_VOX];     // per staged voxel: channels 0 .. 7, then 8 .. 15 (zero)
    const v4s *wsrc = reinterpret_cast<const v4s *>(A.w) + 9 * CH * 4;     // the depth-centre taps
    for (int i = threadIdx.x; i < 9 * CH * 4; i += blockDim.x) wl[i] = wsrc[i];
    for (int i = threadIdx.x; i < RING_VOX; i += blockDim.x) tile[2 * i + 1] = make_uint4(0u, 0u, 0u, 0u);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int T = A.pin.T, S = A.pin.S;
    const int ntx = (A.X + TXW - 1) / TXW, nty = (A.Y + TY - 1) / TY;
    int64_t b = blockIdx.x;
    const int x0 = (int)(b % ntx) * TXW;
    b /= ntx;
    const int y0 = (int)(b % nty) * TY;
    const int si = (int)(b / nty);
    const float4 bias = conv_bias(A, g);
    const int xs = x0 + 16 * wave;
    // the window of time point t0: channel c holds frame clamp(t0 - 2 + c)
    float reg[RING_LD];
    uint32_t w01[RING_LD], w23[RING_LD], w4[RING_LD];   // channels (0, 1), (2, 3), (4, 5 = 0)
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        frame_fetch(A, min(max(t0 - 2 + c, 0), T - 1), si, y0, x0, reg);
#pragma unroll
        for (int k = 0; k < RING_LD; ++k) {
            const uint32_t h = f2bf(reg[k]);
            if (c == 0) w01[k] = h;
            if (c == 1) w01[k] |= h << 16;
            if (c == 2) w23[k] = h;
            if (c == 3) w23[k] |= h << 16;
            if (c == 4) w4[k] = h;
        }
    }
    auto put = [&]() {
#pragma unroll
        for (int k = 0; k < RING_LD; ++k) {
            const int vi = threadIdx.x + 256 * k;
            if (vi < RING_VOX) tile[2 * vi] = make_uint4(w01[k], w23[k], w4[k], 0u);
        }
    };
    put();
    __syncthreads();                         // the weights are staged
    Window<4> win;                           // channels 0 .. 4 carry the input: four taps per MFMA
    win.load(wl, 0, r, g);
    const v4s *tl = reinterpret_cast<const v4s *>(tile);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();                     // the channels of time point t are staged
        const int fn = t + 3;
        if (fn < T) frame_fetch(A, fn, si, y0, x0, reg);
        if (xs < A.X) {
            const int64_t n = (int64_t)t * S + si - (int64_t)A.pin.n0;     // image within the chunk
            for (int ry = 0; ry < TY && y0 + ry < A.Y; ++ry) {
                v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
                win.apply(tl, (ry * TROW + 16 * wave + r) * 4, acc);
                const int y = y0 + ry, xv = xs + r;
                if (xv < A.X) conv_store<EPI_RELU>(A, acc, bias, (n * A.Y + y) * A.X + xv, 0, g);
            }
        }
        if (t + 1 < t1) {
            __syncthreads();                 // every read of time point t's channels is done
            // one time point on: channels shift down by one, frame clamp(t + 3) enters as channel 4
#pragma unroll
            for (int k = 0; k < RING_LD; ++k) {
                w01[k] = (w01[k] >> 16) | (w23[k] << 16);
                w23[k] = (w23[k] >> 16) | (w4[k] << 16);
                if (fn < T) w4[k] = f2bf(reg[k]);
            }
            put();
        }
    }
}

// 3D volumes: a workgroup owns TY3 rows x 64 voxels of ZC3 consecutive z
// slices of one volume and slides along z, keeping the three input slices
// z - 1, z, z + 1 (each with a one-voxel halo in y and x) in an LDS ring; one
// new slice is staged per output slice (16-byte loads, the slice after it
// prefetched into registers), so each input voxel is read about
// (TY3 + 2) / TY3 times instead of 27.
constexpr int TY3 = 4, ZC3 = 16;
constexpr int SL_VOX = (TY3 + 2) * TROW;         // staged voxels per slice
constexpr int SL_U4 = 2 * SL_VOX;                 // 16-byte chunks per slice
constexpr int SL_LD = (SL_U4 + 255) / 256;        // per thread

__device__ __forceinline__ void slice_fetch(const ConvArgs &A, int n, int z, int y0, int x0, uint4 (&reg)[SL_LD])
{
    const uint4 *src = reinterpret_cast<const uint4 *>(A.in);
#pragma unroll
    for (int k = 0; k < SL_LD; ++k) {
        const int idx = threadIdx.x + 256 * k;
        const int row = idx / (2 * TROW), rem = idx - row * (2 * TROW);
        const int gy = y0 - 1 + row, gx = x0 - 1 + (rem >> 1);
        const bool ok = idx < SL_U4 && z >= 0 && z < A.Z && gy >= 0 && gy < A.Y && gx >= 0 && gx < A.X;
        reg[k] = ok ? src[((((int64_t)n * A.Z + z) * A.Y + gy) * A.X + gx) * 2 + (rem & 1)] : make_uint4(0, 0, 0, 0);
    }
}

template <int EPI>
__global__ __launch_bounds__(256) void k_conv3d(const ConvArgs A)
{
    __shared__ v4s wl[TAPS * CH * 4];
    __shared__ uint4 ring[3 * SL_U4];
    const v4s *wsrc = reinterpret_cast<const v4s *>(A.w);
    for (int i = threadIdx.x; i < TAPS * CH * 4; i += blockDim.x) wl[i] = wsrc[i];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int ntx = (A.X + TXW - 1) / TXW, nty = (A.Y + TY3 - 1) / TY3, nzc = (A.Z + ZC3 - 1) / ZC3;
    int64_t t = blockIdx.x;
    const int x0 = (int)(t % ntx) * TXW;
    t /= ntx;
    const int y0 = (int)(t % nty) * TY3;
    t /= nty;
    const int zbeg = (int)(t % nzc) * ZC3;
    const int n = (int)(t / nzc);
    const int zend = min(zbeg + ZC3, A.Z);
    const float4 bias = conv_bias(A, g);
    const int xs = x0 + 16 * wave;           // this wave's segment
    // ring slot of slice z (z >= zbeg - 1)
    auto slot = [&](int z) { return (z - zbeg + 1) % 3; };
    __syncthreads();                         // the weights are staged
    // this lane's weight blocks stay in registers (LDS then serves only the activations):
    // per depth tap dz a 3x3 window of two taps per MFMA (five per window)
    Window<2> win[3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) win[dz].load(wl, dz * 9, r, g);
    uint4 reg[SL_LD];
    slice_fetch(A, n, zbeg - 1, y0, x0, reg);
#pragma unroll
    for (int k = 0; k < SL_LD; ++k) {
        const int idx = threadIdx.x + 256 * k;
        if (idx < SL_U4) ring[slot(zbeg - 1) * SL_U4 + idx] = reg[k];
    }
    slice_fetch(A, n, zbeg, y0, x0, reg);
#pragma unroll
    for (int k = 0; k < SL_LD; ++k) {
        const int idx = threadIdx.x + 256 * k;
        if (idx < SL_U4) ring[slot(zbeg) * SL_U4 + idx] = reg[k];
    }
    slice_fetch(A, n, zbeg + 1, y0, x0, reg);
    const v4s *tl = reinterpret_cast<const v4s *>(ring);
    for (int z = zbeg; z < zend; ++z) {
        __syncthreads();                     // slice z - 2 (the slot of z + 1) is no longer read
#pragma unroll
        for (int k = 0; k < SL_LD; ++k) {
            const int idx = threadIdx.x + 256 * k;
            if (idx < SL_U4) ring[slot(z + 1) * SL_U4 + idx] = reg[k];
        }
        __syncthreads();
        if (z + 2 <= zend) slice_fetch(A, n, z + 2, y0, x0, reg);
        if (xs >= A.X) continue;             // wave-uniform; barriers only at the top of the loop
        for (int ry = 0; ry < TY3 && y0 + ry < A.Y; ++ry) {
            v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
                win[dz].apply(tl, (slot(z - 1 + dz) * SL_VOX + ry * TROW + 16 * wave + r) * 4, acc);
            const int y = y0 + ry, xv = xs + r;
            if (xv < A.X) {
                const int64_t row = ((int64_t)n * A.Z + z) * A.Y + y;
                conv_store<EPI>(A, acc, bias, row * A.X + xv,
                                (int64_t)n * A.v_stride + A.v_off + ((int64_t)z * A.Y + y) * A.X + xv, g);
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

// dW[tap][o][i] = sum_p g[p][o] h[p + tap - 1][i]: M = o, N = i, K = voxels,
// 32 voxels of one x row per MFMA (lane group g takes voxels 8g .. 8g + 7).
__global__ __launch_bounds__(256) void k_wgrad(const WgradArgs A)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int nsx = (A.X + 31) / 32;
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
        const int x0 = xs * 32;
        const int64_t vrow = (((int64_t)n * A.Z + z) * A.Y + y) * A.X;
        v8s ga;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int xv = x0 + 8 * g + j;
            const uint16_t gv = xv < A.X ? A.g[(vrow + xv) * CH + r] : (uint16_t)0;
            ga[j] = (short)gv;
            bsum += bf2f(gv);
        }
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            const int zz = z + dz - 1;
            if (zz < 0 || zz >= A.Z) continue;     // uniform over the wave: zero contribution
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const int yy = y + dy - 1;
                if (yy < 0 || yy >= A.Y) continue;
                const int64_t row = (((int64_t)n * A.Z + zz) * A.Y + yy) * A.X;
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    v8s hb;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int xv = x0 + 8 * g + j;
                        const int xx = xv + dx - 1;
                        hb[j] = (short)((xv < A.X && xx >= 0 && xx < A.X) ? A.h[(row + xx) * CH + r] : (uint16_t)0);
                    }
                    const int tap = (dz * 3 + dy) * 3 + dx;
                    acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, ga),
                                                                       __builtin_bit_cast(v8bf, hb), acc[tap], 0, 0, 0);
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

// grad_flat[layer] <- sum of the per-wave partials, real channels and
// parameter taps only.  A workgroup takes 16 elements; 16 thread groups split
// the partial list into contiguous sixteenths, each thread keeping 8 running
// sums (loads in flight), and the groups are added in order through LDS: a
// fixed summation order, so the gradient is deterministic.
constexpr int WG_RGROUPS = 16;
static_assert((WG_BLOCKS * 4) % (WG_RGROUPS * 8) == 0, "partials split evenly");

__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ part, int nwaves, int layer,
                                                      const NetShape S, float *__restrict__ grad)
{
    __shared__ float red[WG_RGROUPS][17];
    const int el = threadIdx.x & 15, grp = threadIdx.x >> 4;
    const int e = blockIdx.x * 16 + el;
    float acc8[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (e < PART) {
        const int per = nwaves / WG_RGROUPS;
        const float *p = part + (int64_t)grp * per * PART + e;
        for (int w = 0; w < per; w += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) acc8[u] += p[(int64_t)(w + u) * PART];
        }
    }
    red[grp][el] = ((acc8[0] + acc8[1]) + (acc8[2] + acc8[3])) + ((acc8[4] + acc8[5]) + (acc8[6] + acc8[7]));
    __syncthreads();
    if (grp != 0 || e >= PART) return;
    float sum = 0.0f;
    for (int q = 0; q < WG_RGROUPS; ++q) sum += red[q][el];
    const int cin = net_cin(S, layer), cout = COUT[layer];
    if (e < TAPS * CH * CH) {
        const int tap = e / (CH * CH), o = (e / CH) % CH, i = e % CH;
        const int pt = net_ptap(S, tap);
        if (o >= cout || i >= cin || pt < 0) return;
        grad[S.poff[layer] + (o * cin + i) * S.ptaps + pt] = sum;
    } else {
        const int o = e - TAPS * CH * CH;
        if (o >= cout) return;
        grad[S.poff[layer] + cout * cin * S.ptaps + o] = sum;
    }
}

// bf16 weights for the forward ([tap][out][in]) and the input gradient
// (flipped taps, in/out swapped), FP32 biases padded to 16
__global__ void k_pack(const float *__restrict__ master, const NetShape S, uint16_t *__restrict__ wf,
                       uint16_t *__restrict__ wd, float *__restrict__ bias)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 4 * WPACK) return;
    const int layer = e / WPACK, k = e % WPACK;
    const int tap = k / (CH * CH), o = (k / CH) % CH, i = k % CH;
    const int cin = net_cin(S, layer), cout = COUT[layer];
    const float *W = master + S.poff[layer];
    const int pt = net_ptap(S, tap);
    wf[e] = (o < cout && i < cin && pt >= 0) ? f2bf(W[(o * cin + i) * S.ptaps + pt]) : (uint16_t)0;
    // input gradient: out channel o' = forward input i', in channel i' = forward output o'
    const int fpt = net_ptap(S, TAPS - 1 - tap);
    wd[e] = (i < cout && o < cin && fpt >= 0) ? f2bf(W[(i * cin + o) * S.ptaps + fpt]) : (uint16_t)0;
    if (k < CH) bias[layer * CH + k] = k < cout ? master[S.poff[layer] + cout * cin * S.ptaps + k] : 0.0f;
}

// one thread per voxel: its 16 channels (32 bytes) in two 16-byte stores
__global__ void k_pack_input(const PackIn P, int64_t n, int64_t per, uint16_t *__restrict__ h0)
{
    const int cin = P.mode == IN_WARM ? 2 : 5;
    for (int64_t vox = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; vox < n; vox += (int64_t)gridDim.x * blockDim.x) {
        const int64_t img = vox / per, loc = vox - img * per;
        uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int c = 0; c < cin; ++c) {
            const float sc = (P.mode == IN_WARM && c == 1) ? P.inv1 : P.inv0;
            w[c >> 1] |= (uint32_t)f2bf(pack_src(P, img, loc, c, per) * sc) << (16 * (c & 1));
        }
        uint4 *dst = reinterpret_cast<uint4 *>(h0 + vox * CH);
        dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
        dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
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

unsigned grid_of(int64_t work, int per_block)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

struct msf_cnn {
    NetShape shape{};
    int kind = MSF_CNN_WARM_START;
    float cv = 1.0f, cg = 1.0f, co = 1.0f;   // input / feature / output scales (denoiser: cv = c_in)
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
    // two plane sequences of msf_denoise25 (yz and zx planes)
    float *seq = nullptr;
    int64_t seq_cap = 0;
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
                       uint16_t *out_bf, const uint16_t *mask, float *out_f, const float *v, int64_t v_stride,
                       int64_t v_off, float scale, hipStream_t s)
{
    ConvArgs A{in, w, bias, N, Z, Y, X, out_bf, mask, out_f, v, v_stride, v_off, scale, PackIn{}};
    const dim3 block(256);
    if (Z == 1) {
        // depth-1 images: only the depth-centre taps can be non-zero; row tiles staged in LDS
        const int64_t ntile = (int64_t)N * ((Y + TY - 1) / TY) * ((X + TXW - 1) / TXW);
        const dim3 g2((unsigned)std::max<int64_t>(1, std::min<int64_t>(ntile, 4096)));
        switch (epi) {
        case EPI_RELU: hipLaunchKernelGGL((k_conv2d<EPI_RELU, false>), g2, block, 0, s, A); break;
        case EPI_MASK: hipLaunchKernelGGL((k_conv2d<EPI_MASK, false>), g2, block, 0, s, A); break;
        default: hipLaunchKernelGGL((k_conv2d<EPI_RESID, false>), g2, block, 0, s, A); break;
        }
        return hipGetLastError();
    }
    // 3D volumes: z-sliding row tiles
    const int64_t ntile3 = (int64_t)N * ((Z + ZC3 - 1) / ZC3) * ((Y + TY3 - 1) / TY3) * ((X + TXW - 1) / TXW);
    if (ntile3 > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g3((unsigned)ntile3);
    switch (epi) {
    case EPI_RELU: hipLaunchKernelGGL((k_conv3d<EPI_RELU>), g3, block, 0, s, A); break;
    case EPI_MASK: hipLaunchKernelGGL((k_conv3d<EPI_MASK>), g3, block, 0, s, A); break;
    default: hipLaunchKernelGGL((k_conv3d<EPI_RESID>), g3, block, 0, s, A); break;
    }
    return hipGetLastError();
}

// Forward pass of N images [Z][Y][X] whose input channels come from `in`;
// x0 = residual base + c_o f, the base of image n at vbase + n v_stride + v_off.
hipError_t cnn_forward(msf_cnn *C, const PackIn &in, int N, int Z, int Y, int X, const float *vbase, int64_t v_stride,
                       int64_t v_off, float *x0, hipStream_t s, bool keep_input = false)
{
    const int64_t per = (int64_t)Z * Y * X, n = (int64_t)N * per;
    hipError_t e;
    int l0 = 0;
    if (Z == 1 && !keep_input) {
        // depth-1 inference: the first layer stages its input from the FP32 sources
        ConvArgs A{nullptr, C->wf, C->bias, N, Z, Y, X, C->h[1], nullptr, nullptr, nullptr, 0, 0, 0.0f, in};
        const int64_t tiles_per_image = (int64_t)((Y + TY - 1) / TY) * ((X + TXW - 1) / TXW);
        if (in.mode == IN_SEQ && in.n0 % in.S == 0 && N % in.S == 0 && (int64_t)in.S * tiles_per_image <= 0x7fffffff) {
            // whole time points: walk along t with each voxel's five-frame window in registers
            const int t0 = (int)(in.n0 / in.S), t1 = t0 + N / in.S;
            hipLaunchKernelGGL(k_conv2d_first_seq, dim3((unsigned)(in.S * tiles_per_image)), dim3(256), 0, s, A, t0,
                               t1);
        } else {
            const int64_t ntile = (int64_t)N * tiles_per_image;
            const dim3 g2((unsigned)std::max<int64_t>(1, std::min<int64_t>(ntile, 4096)));
            hipLaunchKernelGGL((k_conv2d<EPI_RELU, true>), g2, dim3(256), 0, s, A);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        l0 = 1;
    } else {
        hipLaunchKernelGGL(k_pack_input, dim3(grid_of(n, 256)), dim3(256), 0, s, in, n, per, C->h[0]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int l = l0; l < 3; ++l)
        if ((e = launch_conv(EPI_RELU, C->h[l], C->wf + l * WPACK, C->bias + l * CH, N, Z, Y, X, C->h[l + 1],
                             nullptr, nullptr, nullptr, 0, 0, 0.0f, s)) != hipSuccess)
            return e;
    return launch_conv(EPI_RESID, C->h[3], C->wf + 3 * WPACK, C->bias + 3 * CH, N, Z, Y, X, nullptr, nullptr, x0,
                       vbase, v_stride, v_off, C->co, s);
}

// the input of a caller's images: warm start (v, g) or the denoiser's stacked slices
PackIn caller_input(const msf_cnn *C, const float *v, const float *g)
{
    PackIn P{};
    P.mode = C->kind == MSF_CNN_WARM_START ? IN_WARM : IN_STACK;
    P.a = v;
    P.g = g;
    P.inv0 = 1.0f / C->cv;
    P.inv1 = 1.0f / C->cg;
    return P;
}

hipError_t cnn_pack(msf_cnn *C, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack, dim3((4 * WPACK + 255) / 256), dim3(256), 0, s, C->master, C->shape, C->wf, C->wd,
                       C->bias);
    return hipGetLastError();
}

// [T][Z][Y][X] <-> the plane-k sequence [T][S][H][W]: k = 2 -> [T][X][Z][Y]
// (images (z, y) at fixed x), k = 3 -> [T][Y][Z][X] (images (z, x) at fixed y);
// to = 1: volume -> sequence, to = 0: sequence -> volume
__global__ void k_plane_transpose(const float *__restrict__ in, float *__restrict__ out, int T, int Z, int Y, int X,
                                  int plane, int to)
{
    const int64_t n = (int64_t)T * Z * Y * X;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i;    // volume index [t][z][y][x]
        const int x = (int)(r % X); r /= X;
        const int y = (int)(r % Y); r /= Y;
        const int z = (int)(r % Z);
        const int t = (int)(r / Z);
        const int64_t q = plane == 2 ? (((int64_t)t * X + x) * Z + z) * Y + y : (((int64_t)t * Y + y) * Z + z) * X + x;
        if (to) out[q] = in[i];
        else out[i] = in[q];
    }
}

// plane 2 with coalesced reads and writes: one 32 x 32 (y, x) tile of one
// (t, z) slice per block, through LDS (256 threads = 32 x 8)
__global__ __launch_bounds__(256) void k_transpose_p2(const float *__restrict__ in, float *__restrict__ out, int Z,
                                                      int Y, int X, int to)
{
    __shared__ float tile[32][33];
    const int tz = blockIdx.z, t = tz / Z, z = tz - t * Z;
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t vslice = (int64_t)tz * Y * X;                 // volume [t][z][.][.]
    auto sidx = [&](int x, int y) { return (((int64_t)t * X + x) * Z + z) * Y + y; };   // sequence [t][x][z][y]
    if (to) {
        for (int k = ty; k < 32; k += 8) {
            const int y = by + k, x = bx + tx;
            if (y < Y && x < X) tile[k][tx] = in[vslice + (int64_t)y * X + x];
        }
        __syncthreads();
        for (int k = ty; k < 32; k += 8) {
            const int x = bx + k, y = by + tx;
            if (y < Y && x < X) out[sidx(x, y)] = tile[tx][k];
        }
    } else {
        for (int k = ty; k < 32; k += 8) {
            const int x = bx + k, y = by + tx;
            if (y < Y && x < X) tile[tx][k] = in[sidx(x, y)];
        }
        __syncthreads();
        for (int k = ty; k < 32; k += 8) {
            const int y = by + k, x = bx + tx;
            if (y < Y && x < X) out[vslice + (int64_t)y * X + x] = tile[k][tx];
        }
    }
}

// plane 3: vol [T][Z][Y][X] <-> seq [T][Y][Z][X], x rows stay contiguous:
// one (t, z) slice per block, its Y rows copied as X-long runs
__global__ __launch_bounds__(256) void k_transpose_p3(const float *__restrict__ in, float *__restrict__ out, int Z,
                                                      int Y, int X, int to)
{
    const int tz = blockIdx.x, t = tz / Z, z = tz - t * Z;
    const int n = Y * X;
    const int64_t vslice = (int64_t)tz * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int y = i / X, x = i - y * X;
        const int64_t is = (((int64_t)t * Y + y) * Z + z) * X + x;
        if (to) out[is] = in[vslice + i];
        else out[vslice + i] = in[is];
    }
}

hipError_t plane_transpose(const float *in, float *out, int T, int Z, int Y, int X, int plane, int to, hipStream_t s)
{
    const int64_t slices = (int64_t)T * Z;
    if (plane == 2 && slices <= 65535) {
        const dim3 grid((unsigned)((X + 31) / 32), (unsigned)((Y + 31) / 32), (unsigned)slices);
        hipLaunchKernelGGL(k_transpose_p2, grid, dim3(256), 0, s, in, out, Z, Y, X, to);
    } else if (plane == 3 && (int64_t)Y * X < ((int64_t)1 << 31)) {
        hipLaunchKernelGGL(k_transpose_p3, dim3((unsigned)slices), dim3(256), 0, s, in, out, Z, Y, X, to);
    } else {
        const int64_t n = slices * Y * X;
        hipLaunchKernelGGL(k_plane_transpose, dim3(grid_of(n, 256)), dim3(256), 0, s, in, out, T, Z, Y, X, plane, to);
    }
    return hipGetLastError();
}

// the denoiser on a plane sequence [T][S][H][W] (images chunked so that the
// activations fit in 2^26 voxels); out must not overlap seq
hipError_t denoise_sequence(msf_cnn *C, const float *seq, int T, int S, int H, int W, float *out, hipStream_t s)
{
    const int64_t per = (int64_t)H * W;
    const int64_t N = (int64_t)T * S;
    // chunks of whole time points when S images fit (the first layer then walks along t)
    int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(N, ((int64_t)1 << 26) / per));
    if (chunk >= S) chunk -= chunk % S;
    hipError_t e = cnn_reserve(C, chunk * per);
    if (e != hipSuccess) return e;
    PackIn P{};
    P.mode = IN_SEQ;
    P.a = seq;
    P.T = T;
    P.S = S;
    P.inv0 = 1.0f / C->cv;
    for (int64_t f0 = 0; f0 < N; f0 += chunk) {
        const int nf = (int)std::min<int64_t>(chunk, N - f0);     // a multiple of S when chunk is
        P.n0 = f0;
        e = cnn_forward(C, P, nf, 1, H, W, seq + f0 * per, per, 0, out + f0 * per, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#define CHK(expr)                                            \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

msf_status cnn_create(int kind, const float *params, int64_t n_params, const float *scales, msf_cnn **out)
{
    set_error("");
    const NetShape S = kind == MSF_CNN_WARM_START ? make_shape(2, TAPS) : make_shape(5, 9);
    const int nsc = kind == MSF_CNN_WARM_START ? 3 : 2;
    if (!params || !out || !scales || n_params != S.nparam) {
        set_error(kind == MSF_CNN_WARM_START ? "msf_cnn_create: need 15169 parameters and 3 scales"
                                             : "msf_cnn_create_denoiser: need 5521 parameters and 2 scales");
        return MSF_EINVAL;
    }
    for (int k = 0; k < nsc; ++k)
        if (!(std::isfinite(scales[k]) && scales[k] > 0.0f)) {
            set_error("msf_cnn_create: scales must be positive and finite");
            return MSF_EINVAL;
        }
    for (int64_t i = 0; i < n_params; ++i)
        if (!std::isfinite(params[i])) { set_error("msf_cnn_create: non-finite parameter"); return MSF_EINVAL; }
    msf_cnn *C = new (std::nothrow) msf_cnn();
    if (!C) { set_error("host allocation failed"); return MSF_ENOMEM; }
    C->shape = S;
    C->kind = kind;
    if (kind == MSF_CNN_WARM_START) {
        C->cv = scales[0];
        C->cg = scales[1];
        C->co = scales[2];
    } else {
        C->cv = C->cg = scales[0];
        C->co = scales[1];
    }
    hipError_t e = hipSuccess;
    auto fail = [&](hipError_t err) {
        msf_cnn_destroy(C);
        return hip_fail(err, "msf_cnn_create");
    };
    const int NP = S.nparam;
    if ((e = cnn_alloc(&C->master, NP)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->m, NP)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->v, NP)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->grad, NP)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->wf, 4 * WPACK)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->wd, 4 * WPACK)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->bias, 4 * CH)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->part, (size_t)WG_BLOCKS * 4 * PART)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->lpart, 65536)) != hipSuccess) return fail(e);
    if ((e = cnn_alloc(&C->flag, 4)) != hipSuccess) return fail(e);
    if ((e = hipHostMalloc((void **)&C->hlpart, 65536 * sizeof(double), hipHostMallocDefault)) != hipSuccess) return fail(e);
    if ((e = hipMemcpy(C->master, params, NP * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
    if ((e = hipMemset(C->m, 0, NP * sizeof(float))) != hipSuccess) return fail(e);
    if ((e = hipMemset(C->v, 0, NP * sizeof(float))) != hipSuccess) return fail(e);
    if ((e = hipMemset(C->grad, 0, NP * sizeof(float))) != hipSuccess) return fail(e);
    if ((e = cnn_pack(C, nullptr)) != hipSuccess) return fail(e);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(e);
    *out = C;
    return MSF_OK;
}

bool shape_ok(const msf_cnn *C, int32_t n, int32_t nz, int32_t ny, int32_t nx)
{
    if (n <= 0 || nz <= 0 || ny <= 0 || nx <= 0) return false;
    return C->kind == MSF_CNN_WARM_START || nz == 1;
}

}  // namespace

int cnn_kind(const msf_cnn *C) { return C->kind; }

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
    // images are independent: evaluate them in chunks of at most 2^26 voxels
    // (activations take 32 bytes per voxel and layer)
    const int64_t per = (int64_t)Z * Y * X;
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(N, ((int64_t)1 << 26) / per));
    hipError_t e = cnn_reserve(C, (int64_t)chunk * per);
    if (e != hipSuccess) return e;
    const bool stack = C->kind == MSF_CNN_DENOISER;
    const int64_t in_img = stack ? 5 * per : per;     // input floats per image
    for (int f0 = 0; f0 < N; f0 += chunk) {
        const int nf = std::min(chunk, N - f0);
        const PackIn P = caller_input(C, v + f0 * in_img, stack ? nullptr : g + f0 * per);
        e = cnn_forward(C, P, nf, Z, Y, X, v + f0 * in_img, in_img, stack ? 2 * per : 0, x0 + f0 * per, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t denoise25_internal(msf_cnn *C, const float *w, int T, int Z, int Y, int X, int plane, float *out,
                              float *scratch_a, float *scratch_b, hipStream_t s)
{
    if (plane == 1) return denoise_sequence(C, w, T, Z, Y, X, out, s);
    hipError_t e = plane_transpose(w, scratch_a, T, Z, Y, X, plane, 1, s);
    if (e != hipSuccess) return e;
    e = plane == 2 ? denoise_sequence(C, scratch_a, T, X, Z, Y, scratch_b, s)
                   : denoise_sequence(C, scratch_a, T, Y, Z, X, scratch_b, s);
    if (e != hipSuccess) return e;
    return plane_transpose(scratch_b, out, T, Z, Y, X, plane, 0, s);
}

extern "C" {

msf_status msf_cnn_create(const float *params, int64_t n_params, const float *scales, msf_cnn **out)
{
    return cnn_create(MSF_CNN_WARM_START, params, n_params, scales, out);
}

msf_status msf_cnn_create_denoiser(const float *params, int64_t n_params, const float *scales, msf_cnn **out)
{
    return cnn_create(MSF_CNN_DENOISER, params, n_params, scales, out);
}

void msf_cnn_destroy(msf_cnn *C)
{
    if (!C) return;
    (void)hipDeviceSynchronize();
    cnn_free_ws(C);
    void *ps[] = {C->master, C->m, C->v, C->grad, C->wf, C->wd, C->bias, C->part, C->lpart, C->flag, C->io, C->seq};
    for (void *q : ps)
        if (q) (void)hipFree(q);
    if (C->hlpart) (void)hipHostFree(C->hlpart);
    delete C;
}

int32_t msf_cnn_kind(const msf_cnn *C) { return C ? C->kind : -1; }

int64_t msf_cnn_n_params(const msf_cnn *C) { return C ? C->shape.nparam : 0; }

msf_status msf_cnn_get_params(const msf_cnn *C, float *params)
{
    if (!C || !params) { set_error("null argument"); return MSF_EINVAL; }
    CHK(hipMemcpy(params, C->master, C->shape.nparam * sizeof(float), hipMemcpyDeviceToHost));
    return MSF_OK;
}

msf_status msf_cnn_infer(msf_cnn *C, const float *v, const float *g, int32_t n, int32_t nz, int32_t ny, int32_t nx,
                         float *x0, void *stream)
{
    set_error("");
    if (!C || !v || !x0 || (C->kind == MSF_CNN_WARM_START && !g) || !shape_ok(C, n, nz, ny, nx)) {
        set_error("invalid argument (the denoiser takes images with nz = 1)");
        return MSF_EINVAL;
    }
    CHK(cnn_infer_internal(C, v, g, n, nz, ny, nx, x0, (hipStream_t)stream));
    return MSF_OK;
}

msf_status msf_denoise25(msf_cnn *C, const float *w, int32_t n_frames, int32_t nz, int32_t ny, int32_t nx,
                         int32_t plane, float *out, void *stream)
{
    set_error("");
    if (!C || !w || !out || C->kind != MSF_CNN_DENOISER || n_frames <= 0 || nz <= 0 || ny <= 0 || nx <= 0 ||
        plane < 1 || plane > 3) {
        set_error("msf_denoise25: needs a denoiser network, a non-empty [n_frames][nz][ny][nx] volume, plane 1..3");
        return MSF_EINVAL;
    }
    const int64_t n = (int64_t)n_frames * nz * ny * nx;
    const uintptr_t wb = (uintptr_t)w, ob = (uintptr_t)out, bytes = (uintptr_t)n * sizeof(float);
    if (wb < ob + bytes && ob < wb + bytes) { set_error("msf_denoise25: out overlaps w"); return MSF_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    float *sa = nullptr, *sb = nullptr;
    if (plane != 1) {
        // the network keeps two sequence volumes; a larger volume replaces them
        if (n > C->seq_cap) {
            if (C->seq) {
                CHK(hipStreamSynchronize(s));
                (void)hipFree(C->seq);
            }
            C->seq = nullptr;
            C->seq_cap = 0;
            CHK(cnn_alloc(&C->seq, (size_t)(2 * n)));
            C->seq_cap = n;
        }
        sa = C->seq;
        sb = C->seq + n;
    }
    CHK(denoise25_internal(C, w, n_frames, nz, ny, nx, plane, out, sa, sb, s));
    return MSF_OK;
}

msf_status msf_cnn_train_step(msf_cnn *C, const float *v, const float *g, const float *target, int32_t n, int32_t nz,
                              int32_t ny, int32_t nx, double lr, int32_t apply, double *loss_out, float *grad_out,
                              void *stream)
{
    set_error("");
    if (!C || !v || !target || (C->kind == MSF_CNN_WARM_START && !g) || !shape_ok(C, n, nz, ny, nx) || !(lr >= 0.0)) {
        set_error("invalid argument (the denoiser takes images with nz = 1)");
        return MSF_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t per = (int64_t)nz * ny * nx;
    const int64_t nvox = (int64_t)n * per;
    const bool stack = C->kind == MSF_CNN_DENOISER;
    CHK(cnn_reserve(C, nvox));
    CHK(cnn_forward(C, caller_input(C, v, g), n, nz, ny, nx, v, stack ? 5 * per : per, stack ? 2 * per : 0, C->pred,
                    s, true));
    const unsigned lb = grid_of(nvox, 256);
    hipLaunchKernelGGL(k_mse, dim3(lb), dim3(256), 0, s, C->pred, target, nvox, C->co, C->ga, C->lpart);
    CHK(hipGetLastError());
    // backward: g_l is the gradient at layer l's output (bf16, ReLU mask applied)
    uint16_t *gcur = C->ga, *gnext = C->gb;
    for (int l = 3; l >= 0; --l) {
        WgradArgs W{gcur, C->h[l], n, nz, ny, nx, C->part};
        hipLaunchKernelGGL(k_wgrad, dim3(WG_BLOCKS), dim3(256), 0, s, W);
        CHK(hipGetLastError());
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((PART + 15) / 16), dim3(256), 0, s, C->part, WG_BLOCKS * 4, l,
                           C->shape, C->grad);
        CHK(hipGetLastError());
        if (l > 0) {
            CHK(launch_conv(EPI_MASK, gcur, C->wd + l * WPACK, nullptr, n, nz, ny, nx, gnext, C->h[l], nullptr,
                            nullptr, 0, 0, 0.0f, s));
            std::swap(gcur, gnext);
        }
    }
    const int NP = C->shape.nparam;
    CHK(hipMemcpyAsync(C->hlpart, C->lpart, lb * sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad_out) CHK(hipMemcpyAsync(grad_out, C->grad, NP * sizeof(float), hipMemcpyDeviceToHost, s));
    if (apply) {
        C->step++;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - std::pow(b1, (float)C->step), c2 = 1.0f - std::pow(b2, (float)C->step);
        hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, s, C->master, C->m, C->v, C->grad, NP,
                           (float)lr, b1, b2, 1e-8f, c1, c2);
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
