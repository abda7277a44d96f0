// Learned initial guess for the Poisson solve (Sec. 2.1, Eqs. (3)-(4);
// multigrid of Sec. 4): a small 3D U-Net maps the scaled charge density and
// the electrode ramp to the scaled potential.  Not part of the paper's
// method; the multigrid solve that follows still decides convergence.
//
// Layout: activations are channels-last, [cell][channel] with the channel
// stride padded to a power of two >= 8, stored as bfloat16; gradients are
// FP32 in the same layout.  A 3x3x3 convolution is an implicit GEMM
// (M = cells, N = output channels, K = 27 taps x input channels) on
// v_mfma_f32_16x16x32_bf16: a workgroup owns a 16 x 8 x 2 block of cells x
// up to 64 output channels and stages the block's input halo in LDS, 16
// channels at a time; K advances 32 at a time (a lane's 8 K values are 8
// consecutive channels of one tap: one 16-byte LDS read), FP32
// accumulation, bias and ReLU fused into the store.  The input gradient is
// the same kernel on the FP32 output gradient with flipped, transposed
// weights; weight gradients are an FP32 reduction over cells in
// fixed-order chunks (deterministic).
#include "vd_internal.hpp"

namespace vd {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

// FP32 -> bfloat16, round to nearest even (finite inputs)
__host__ __device__ __forceinline__ u16 f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    return (u16)u;
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }
// the same rounding (to nearest even) by the conversion instruction
__device__ __forceinline__ u16 f2bf_hw(float f) { return __builtin_bit_cast(u16, (__bf16)f); }
__device__ __forceinline__ uint32_t f2bf2_hw(float lo, float hi) {
    return (uint32_t)f2bf_hw(lo) | ((uint32_t)f2bf_hw(hi) << 16);
}

constexpr int kConvWaves = 4;             // wavefronts per workgroup, 32 cells each

struct ConvArgs {
    const void *in;       // [cell][cin_s], bf16 or FP32
    int cin_s;
    int nx, ny, nz;
    const u16 *w;         // packed [cop][nch][28][16] bf16
    const float *bias;    // [co] or null
    void *out;            // [cell][out_s], bf16 or FP32
    int out_f32, out_s, co, relu;
};

// Tile of the convolution: 16 x 8 x 2 output cells (16 MFMA row blocks of
// 16 cells along x, four per wavefront), its input halo 18 x 10 x 4 cells
// staged in LDS 16 channels at a time (32 bytes per cell).  A K step of 32
// covers two taps x 16 channels; 27 taps are padded to 28 (the padded tap's
// weights are zero and its operand is read from a valid slot).
constexpr int kTX = 16, kTY = 8, kTZ = 2;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHalo = kHX * kHY * kHZ;

// LDS slot (in 16-byte units) of half h (channels 8h..8h+7) of halo cell
// c: the two halves in separate planes, so that the 16-byte reads of
// consecutive cells are consecutive slots
__device__ __forceinline__ int lds_slot(int c, int h) { return h * kHalo + c; }
// halo offset of tap t (dz, dy, dx = t / 9, t / 3 % 3, t % 3)
__host__ __device__ constexpr int tap_off(int t) { return t % 3 + kHX * ((t / 3) % 3 + kHY * (t / 9)); }

// Weights of a chunk sit in LDS as [column][28 taps x 2 halves] 16-byte
// slots with one slot of padding per column, so that the 16 columns read
// by one K step fall in different banks.
constexpr int kWRow = 57;

template <int NB, bool IN_F32>
__global__ void __launch_bounds__(64 * kConvWaves) k_conv(ConvArgs a) {
    __shared__ u32x4 xs[2 * kHalo];
    __shared__ u32x4 wl[NB * 16 * kWRow];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int ntx = (nx + kTX - 1) / kTX, nty = (ny + kTY - 1) / kTY;
    const int bt = blockIdx.x;
    const int x0 = (bt % ntx) * kTX, y0 = ((bt / ntx) % nty) * kTY, z0 = (bt / (ntx * nty)) * kTZ;
    const int col0 = blockIdx.y * NB * 16;          // first output column of this workgroup
    f32x4 acc[4][NB];
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
        for (int nb = 0; nb < NB; nb++) acc[q][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the wavefront's rows: y = 4 (wave & 1) + q, z = wave >> 1
    const int ry = 4 * (wave & 1), rz = wave >> 1;
    const int nch = (a.cin_s + 15) >> 4;
    constexpr int kNT = 64 * kConvWaves;
    constexpr int kHalf = (2 * kHalo + kNT - 1) / kNT;          // halo items per thread
    constexpr int kWIt = (NB * 16 * 56 + kNT - 1) / kNT;        // weight items per thread
    for (int ch = 0; ch < nch; ch++) {
        // every load of the chunk is issued before the first LDS store
        u32x4 hv[kHalf], wv[kWIt];
        {
            // item it = threadIdx + u kNT is half h = it & 1 (fixed per
            // thread) of halo cell it >> 1, which advances by kNT / 2 cells
            // per u: the halo coordinates are stepped, not divided
            const int h = threadIdx.x & 1, c0 = ch * 16 + h * 8;
            int c = threadIdx.x >> 1;
            int hx = c % kHX, hy = (c / kHX) % kHY, hz = c / (kHX * kHY);
            constexpr int kStep = kNT / 2, kSx = kStep % kHX, kSy = (kStep / kHX) % kHY;
            static_assert(kStep < kHX * kHY, "halo step");
#pragma unroll
            for (int u = 0; u < kHalf; u++) {
                const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
                hv[u] = u32x4{0u, 0u, 0u, 0u};
                if (c < kHalo && (unsigned)gx < (unsigned)nx && (unsigned)gy < (unsigned)ny && (unsigned)gz < (unsigned)nz &&
                    c0 < a.cin_s) {
                    const unsigned off = ((unsigned)(gz * ny + gy) * (unsigned)nx + (unsigned)gx) * (unsigned)a.cin_s + c0;
                    if (!IN_F32) {
                        hv[u] = gld((const u32x4 *)((const u16 *)a.in + off), 0);
                    } else {
                        const f32x4 *pp = (const f32x4 *)((const float *)a.in + off);
                        const f32x4 lo = gld(pp, 0), hi = gld(pp, 1);
                        hv[u] = u32x4{f2bf2_hw(lo[0], lo[1]), f2bf2_hw(lo[2], lo[3]), f2bf2_hw(hi[0], hi[1]),
                                      f2bf2_hw(hi[2], hi[3])};
                    }
                }
                c += kStep;
                hx += kSx;
                hy += kSy;
                if (hx >= kHX) { hx -= kHX; hy += 1; }
                if (hy >= kHY) { hy -= kHY; hz += 1; }
            }
        }
        const u32x4 *wg = (const u32x4 *)a.w;
#pragma unroll
        for (int u = 0; u < kWIt; u++) {
            const int it = threadIdx.x + u * kNT;
            const int n = it / 56, j = it - n * 56;
            if (it < NB * 16 * 56) wv[u] = gld(wg, ((long)(col0 + n) * nch + ch) * 56 + j);
        }
        if (ch) __syncthreads();     // the previous chunk's reads are done
#pragma unroll
        for (int u = 0; u < kHalf; u++) {
            const int it = threadIdx.x + u * kNT;
            if (it < 2 * kHalo) xs[lds_slot(it >> 1, it & 1)] = hv[u];
        }
#pragma unroll
        for (int u = 0; u < kWIt; u++) {
            const int it = threadIdx.x + u * kNT;
            const int n = it / 56, j = it - n * 56;
            if (it < NB * 16 * 56) wl[n * kWRow + j] = wv[u];
        }
        __syncthreads();
        // K step st: lanes kq < 2 take tap 2 st, kq >= 2 tap 2 st + 1 (tap
        // 27 reads tap 26's slot, its weights are zero); fragments of step
        // st + 1 are read while step st multiplies
        const int hsel = kq >> 1;
        const int lb = lds_slot(r + kHX * (ry + kHY * rz), kq & 1);
        int wb[NB];
#pragma unroll
        for (int nb = 0; nb < NB; nb++) wb[nb] = (nb * 16 + r) * kWRow + (kq & 1) + 2 * hsel;
        bf16x8 A[2][4], B[2][NB];
        auto load = [&](int st, int buf) {
            const int t0 = 2 * st, t1 = 2 * st + 1 < 27 ? 2 * st + 1 : 26;
            const int base = lb + (hsel ? tap_off(t1) : tap_off(t0));
#pragma unroll
            for (int nb = 0; nb < NB; nb++) B[buf][nb] = __builtin_bit_cast(bf16x8, wl[wb[nb] + 4 * st]);
#pragma unroll
            for (int q = 0; q < 4; q++) A[buf][q] = __builtin_bit_cast(bf16x8, xs[base + q * kHX]);
        };
        load(0, 0);
#pragma unroll
        for (int st = 0; st < 14; st++) {
            if (st + 1 < 14) load(st + 1, (st + 1) & 1);
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int nb = 0; nb < NB; nb++)
                    acc[q][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[st & 1][q], B[st & 1][nb], acc[q][nb], 0, 0, 0);
        }
    }
    // lane holds rows 4 kq .. 4 kq + 3 (cells along x) of column r (output channel)
    const bool fullx = x0 + kTX <= nx;
    float bv[NB];
#pragma unroll
    for (int nb = 0; nb < NB; nb++) {
        const int col = col0 + nb * 16 + r;
        bv[nb] = (a.bias && col < a.co) ? gld(a.bias, col) : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int gy = y0 + ry + q, gz = z0 + rz;
        if (gy >= ny || gz >= nz) continue;
        const unsigned rowc = (unsigned)(gz * ny + gy) * (unsigned)nx + (unsigned)(x0 + 4 * kq);
#pragma unroll
        for (int nb = 0; nb < NB; nb++) {
            const int col = col0 + nb * 16 + r;
            if (col >= a.out_s) continue;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                if (!fullx && x0 + 4 * kq + e >= nx) continue;
                const unsigned o = (rowc + e) * (unsigned)a.out_s + col;
                float val = 0.0f;
                if (col < a.co) {
                    val = acc[q][nb][e] + bv[nb];
                    if (a.relu) val = fmaxf(val, 0.0f);
                }
                if (a.out_f32) gst((float *)a.out, o, val);
                else gst((u16 *)a.out, o, f2bf_hw(val));
            }
        }
    }
}

// The same convolution for inputs of at most 16 channels (one chunk), with
// the workgroup marching along z: it owns a 16 x 8 column of kZS slabs of
// two output planes, keeps four input halo planes in an LDS ring (plane k
// of the march, z = z0 - 1 + k, in slot k % 4), stages the weights once,
// and loads the next slab's two new planes into registers while the
// current slab multiplies.
constexpr int kZS = 4;
constexpr int kPlane = kHX * kHY;                 // halo cells per plane

template <int NB, bool IN_F32>
__global__ void __launch_bounds__(64 * kConvWaves) k_conv_z(ConvArgs a) {
    __shared__ u32x4 xs[2 * 4 * kPlane];          // [half][slot][halo cell of the plane]
    __shared__ u32x4 wl[NB * 16 * kWRow];
    constexpr int kNT = 64 * kConvWaves;
    constexpr int kPIt = (2 * 2 * kPlane + kNT - 1) / kNT;   // items of two planes per thread
    constexpr int kWIt = (NB * 16 * 56 + kNT - 1) / kNT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int ntx = (nx + kTX - 1) / kTX, nty = (ny + kTY - 1) / kTY;
    const int bt = blockIdx.x;
    const int x0 = (bt % ntx) * kTX, y0 = ((bt / ntx) % nty) * kTY, z0 = (bt / (ntx * nty)) * (2 * kZS);
    const int col0 = blockIdx.y * NB * 16;
    // this thread's items of a pair of planes: item it = threadIdx + u kNT,
    // half h = it & 1, cell it >> 1 of the pair (plane it >> 1 >= kPlane)
    const int h = threadIdx.x & 1, c0 = h * 8;
    auto load_pair = [&](int k0, u32x4 *v) {          // planes k0, k0 + 1 of the march
#pragma unroll
        for (int u = 0; u < kPIt; u++) {
            const int c = (threadIdx.x + u * kNT) >> 1;
            const int pl = c >= kPlane ? 1 : 0, cc = c - pl * kPlane;
            const int hx = cc % kHX, hy = cc / kHX;
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 - 1 + k0 + pl;
            v[u] = u32x4{0u, 0u, 0u, 0u};
            if (c < 2 * kPlane && (unsigned)gx < (unsigned)nx && (unsigned)gy < (unsigned)ny && (unsigned)gz < (unsigned)nz &&
                c0 < a.cin_s) {
                const unsigned off = ((unsigned)(gz * ny + gy) * (unsigned)nx + (unsigned)gx) * (unsigned)a.cin_s + c0;
                if (!IN_F32) {
                    v[u] = gld((const u32x4 *)((const u16 *)a.in + off), 0);
                } else {
                    const f32x4 *pp = (const f32x4 *)((const float *)a.in + off);
                    const f32x4 lo = gld(pp, 0), hi = gld(pp, 1);
                    v[u] = u32x4{f2bf2_hw(lo[0], lo[1]), f2bf2_hw(lo[2], lo[3]), f2bf2_hw(hi[0], hi[1]), f2bf2_hw(hi[2], hi[3])};
                }
            }
        }
    };
    auto store_pair = [&](int k0, const u32x4 *v) {
#pragma unroll
        for (int u = 0; u < kPIt; u++) {
            const int c = (threadIdx.x + u * kNT) >> 1;
            if (c < 2 * kPlane) {
                const int pl = c >= kPlane ? 1 : 0, cc = c - pl * kPlane;
                xs[(h * 4 + ((k0 + pl) & 3)) * kPlane + cc] = v[u];
            }
        }
    };
    {
        u32x4 p0[kPIt], p1[kPIt], wv[kWIt];
        load_pair(0, p0);
        load_pair(2, p1);
        const u32x4 *wg = (const u32x4 *)a.w;
#pragma unroll
        for (int u = 0; u < kWIt; u++) {
            const int it = threadIdx.x + u * kNT;
            const int n = it / 56, j = it - n * 56;
            if (it < NB * 16 * 56) wv[u] = gld(wg, (long)(col0 + n) * 56 + j);
        }
        store_pair(0, p0);
        store_pair(2, p1);
#pragma unroll
        for (int u = 0; u < kWIt; u++) {
            const int it = threadIdx.x + u * kNT;
            const int n = it / 56, j = it - n * 56;
            if (it < NB * 16 * 56) wl[n * kWRow + j] = wv[u];
        }
        __syncthreads();
    }
    const int ry = 4 * (wave & 1), rz = wave >> 1;
    const int hsel = kq >> 1;
    const int lxy = r + kHX * ry;                 // the lane's cell within a plane (row q adds q kHX)
    int wb[NB];
#pragma unroll
    for (int nb = 0; nb < NB; nb++) wb[nb] = (nb * 16 + r) * kWRow + (kq & 1) + 2 * hsel;
    float bv[NB];
#pragma unroll
    for (int nb = 0; nb < NB; nb++) {
        const int col = col0 + nb * 16 + r;
        bv[nb] = (a.bias && col < a.co) ? gld(a.bias, col) : 0.0f;
    }
    const bool fullx = x0 + kTX <= nx;
    for (int sl = 0; sl < kZS; sl++) {
        const int zs = z0 + 2 * sl;                  // first output plane of the slab
        if (zs >= nz) break;
        u32x4 nxt[kPIt];
        const bool more = sl + 1 < kZS && zs + 2 < nz;
        if (more) load_pair(2 * sl + 4, nxt);
        f32x4 acc[4][NB];
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int nb = 0; nb < NB; nb++) acc[q][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        // input plane of row rz, tap dz: march plane 2 sl + rz + dz, slot (2 sl + rz + dz) & 3
        bf16x8 A[2][4], B[2][NB];
        auto load = [&](int st, int buf) {
            const int t0 = 2 * st, t1 = 2 * st + 1 < 27 ? 2 * st + 1 : 26;
            const int t = hsel ? t1 : t0;
            const int dz = hsel ? t1 / 9 : t0 / 9;
            const int xy = hsel ? (t1 % 3 + kHX * ((t1 / 3) % 3)) : (t0 % 3 + kHX * ((t0 / 3) % 3));
            const int base = ((kq & 1) * 4 + ((2 * sl + rz + dz) & 3)) * kPlane + lxy + xy;
            (void)t;
#pragma unroll
            for (int nb = 0; nb < NB; nb++) B[buf][nb] = __builtin_bit_cast(bf16x8, wl[wb[nb] + 4 * st]);
#pragma unroll
            for (int q = 0; q < 4; q++) A[buf][q] = __builtin_bit_cast(bf16x8, xs[base + q * kHX]);
        };
        load(0, 0);
#pragma unroll
        for (int st = 0; st < 14; st++) {
            if (st + 1 < 14) load(st + 1, (st + 1) & 1);
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int nb = 0; nb < NB; nb++)
                    acc[q][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[st & 1][q], B[st & 1][nb], acc[q][nb], 0, 0, 0);
        }
        const int gz = zs + rz;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int gy = y0 + ry + q;
            if (gy >= ny || gz >= nz) continue;
            const unsigned rowc = (unsigned)(gz * ny + gy) * (unsigned)nx + (unsigned)(x0 + 4 * kq);
#pragma unroll
            for (int nb = 0; nb < NB; nb++) {
                const int col = col0 + nb * 16 + r;
                if (col >= a.out_s) continue;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    if (!fullx && x0 + 4 * kq + e >= nx) continue;
                    const unsigned o = (rowc + e) * (unsigned)a.out_s + col;
                    float val = 0.0f;
                    if (col < a.co) {
                        val = acc[q][nb][e] + bv[nb];
                        if (a.relu) val = fmaxf(val, 0.0f);
                    }
                    if (a.out_f32) gst((float *)a.out, o, val);
                    else gst((u16 *)a.out, o, f2bf_hw(val));
                }
            }
        }
        if (more) {
            __syncthreads();                        // slots of planes 2 sl, 2 sl + 1 are free
            store_pair(2 * sl + 4, nxt);
            __syncthreads();
        }
    }
}

// packed bf16 weights of one convolution, in 16-channel chunks of the
// input: forward [cop][nch][28][16] with element (n, q, tap, c) =
// w[n][tap][16 q + c]; transposed (for the input gradient)
// [cipT][nchT][28][16] with element (n, q, tap', c) = w[16 q + c][26 - tap'][n]
__global__ void k_pack(const float *__restrict__ w, int ci, int co, int nch, int cop, u16 *__restrict__ wf, int nchT, int cipT,
                       u16 *__restrict__ wt) {
    const long n1 = (long)cop * nch * 448, n2 = (long)cipT * nchT * 448;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n1 + n2; q += (long)gridDim.x * blockDim.x) {
        if (q < n1) {
            const int n = (int)(q / (nch * 448)), rem = (int)(q % (nch * 448));
            const int tap = (rem % 448) / 16, c = (rem / 448) * 16 + rem % 16;
            float v = 0.0f;
            if (n < co && c < ci && tap < 27) v = gld(w, ((long)n * 27 + tap) * ci + c);
            gst(wf, q, f2bf(v));
        } else {
            const long q2 = q - n1;
            const int n = (int)(q2 / (nchT * 448)), rem = (int)(q2 % (nchT * 448));
            const int tp = (rem % 448) / 16, c = (rem / 448) * 16 + rem % 16;
            float v = 0.0f;
            if (n < ci && c < co && tp < 27) v = gld(w, ((long)c * 27 + (26 - tp)) * ci + n);
            gst(wt, q2, f2bf(v));
        }
    }
}

// Weight and bias gradient partials on v_mfma_f32_16x16x4_f32: workgroup
// (chunk, block pair) owns a 16 output-channel x 16 input-channel block of
// all 27 taps (K = cells, 4 per step; a lane's operand is one value, so the
// channels-last layouts need no transposition).  Its chunk is a run of the
// convolution's 16 x 8 x 2 cell blocks: the output gradient of a block
// (FP32) and the input halo (bf16) are staged in LDS, wavefront w
// accumulates taps w, w + 4, ...; the sums run in a fixed order
// (deterministic).  Block-pair 0 (first block of each) also sums the
// output gradient per channel for the bias.
struct WgArgs {
    const u16 *x;         // [cell][xs] bf16, channels >= ci ignored
    int xs, ci;
    const float *dy;      // [cell][dys] FP32, channels >= co ignored
    int dys, co;
    int nx, ny, nz;
    int tiles_per_chunk;
    float *part, *partb;
};

typedef float f32x4v __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_wgrad(WgArgs a) {
    __shared__ __align__(16) float dyl[kTX * kTY * kTZ * 16];
    __shared__ __align__(16) u16 xl[kHalo * 16];
    __shared__ float bred[256 * 4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int ntx = (nx + kTX - 1) / kTX, nty = (ny + kTY - 1) / kTY, ntz = (nz + kTZ - 1) / kTZ;
    const int ntiles = ntx * nty * ntz;
    const int ncb = (a.co + 15) / 16;
    const int cb = blockIdx.y % ncb, ib = blockIdx.y / ncb;
    const int t_begin = blockIdx.x * a.tiles_per_chunk;
    const int t_end = min(t_begin + a.tiles_per_chunk, ntiles);
    f32x4v acc[7];
#pragma unroll
    for (int i = 0; i < 7; i++) acc[i] = f32x4v{0.f, 0.f, 0.f, 0.f};
    float bsum[4] = {0.f, 0.f, 0.f, 0.f};     // channels cb 16 + 4 (threadIdx & 3) + m
    for (int t = t_begin; t < t_end; t++) {
        const int x0 = (t % ntx) * kTX, y0 = ((t / ntx) % nty) * kTY, z0 = (t / (ntx * nty)) * kTZ;
        // every load of the block is issued before the first LDS store:
        // the output gradient as 4-channel quads ([cell][4 quads] FP32), the
        // input halo as 8-channel halves ([halo cell][2 halves] bf16);
        // channels past co (ci) read as zero
        constexpr int kDq = kTX * kTY * kTZ * 4 / 256, kXh = (2 * kHalo + 255) / 256;
        f32x4 dq[kDq];
        u32x4 xh[kXh];
#pragma unroll
        for (int u = 0; u < kDq; u++) {
            const int e = threadIdx.x + 256 * u;
            const int c = e >> 2, k = 4 * (e & 3);
            const int gx = x0 + (c % kTX), gy = y0 + (c / kTX) % kTY, gz = z0 + c / (kTX * kTY);
            dq[u] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (gx < nx && gy < ny && gz < nz && cb * 16 + k + 4 <= a.dys)
                dq[u] = gld((const f32x4 *)(a.dy + (gx + nx * (gy + (long)ny * gz)) * a.dys + cb * 16 + k), 0);
#pragma unroll
            for (int m = 0; m < 4; m++)
                if (cb * 16 + k + m >= a.co) dq[u][m] = 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kXh; u++) {
            const int e = threadIdx.x + 256 * u;
            const int c = e >> 1, k = 8 * (e & 1);
            const int gx = x0 + (c % kHX) - 1, gy = y0 + (c / kHX) % kHY - 1, gz = z0 + c / (kHX * kHY) - 1;
            xh[u] = u32x4{0u, 0u, 0u, 0u};
            if (e < 2 * kHalo && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz && ib * 16 + k + 8 <= a.xs)
                xh[u] = gld((const u32x4 *)(a.x + (gx + nx * (gy + (long)ny * gz)) * a.xs + ib * 16 + k), 0);
#pragma unroll
            for (int m = 0; m < 8; m++)
                if (ib * 16 + k + m >= a.ci) xh[u][m >> 1] &= (m & 1) ? 0x0000FFFFu : 0xFFFF0000u;
        }
        if (t > t_begin) __syncthreads();     // the previous block's reads are done
#pragma unroll
        for (int u = 0; u < kDq; u++) {
            const int e = threadIdx.x + 256 * u;
            *(f32x4 *)&dyl[4 * e] = dq[u];
#pragma unroll
            for (int m = 0; m < 4; m++) bsum[m] += dq[u][m];
        }
#pragma unroll
        for (int u = 0; u < kXh; u++) {
            const int e = threadIdx.x + 256 * u;
            if (e < 2 * kHalo) *(u32x4 *)&xl[8 * e] = xh[u];
        }
        __syncthreads();
        // K step st: the lane's cell is c = 4 st + kg, at halo position
        // kg + (4 (st % 4) + kHX ((st / 4) % 8 + kHY (st / 32))) + tap offset
#pragma unroll 4
        for (int st = 0; st < kTX * kTY * kTZ / 4; st++) {
            const float Av = dyl[(4 * st + kg) * 16 + col];
            const int hb = kg + 4 * (st % 4) + kHX * ((st / 4) % kTY + kHY * (st / (4 * kTY)));
            float Bv[7];
#pragma unroll
            for (int i = 0; i < 7; i++) {
                const int tap = wave + 4 * i < 27 ? wave + 4 * i : 26;
                Bv[i] = bf2f(xl[(hb + tap_off(tap)) * 16 + col]);
            }
#pragma unroll
            for (int i = 0; i < 7; i++)
                if (wave + 4 * i < 27) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(Av, Bv[i], acc[i], 0, 0, 0);
        }
    }
    // lane holds rows 4 kg .. 4 kg + 3 (output channels) of column col (input channel)
    const int nout = a.ci * a.co;
    const int ic = ib * 16 + col;
#pragma unroll
    for (int i = 0; i < 7; i++) {
        const int tap = wave + 4 * i;
        if (tap >= 27 || ic >= a.ci) continue;
        float *out = a.part + ((long)blockIdx.x * 27 + tap) * nout;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int oc = cb * 16 + 4 * kg + e;
            if (oc < a.co) gst(out, oc * a.ci + ic, acc[i][e]);
        }
    }
    if (ib == 0) {
        // fixed-order sum over the 64 threads of each channel quad
#pragma unroll
        for (int m = 0; m < 4; m++) bred[threadIdx.x * 4 + m] = bsum[m];
        __syncthreads();
        const int k = threadIdx.x;
        if (k < 16 && cb * 16 + k < a.co) {
            float sacc = 0.0f;
            for (int q = 0; q < 64; q++) sacc += bred[(4 * q + (k >> 2)) * 4 + (k & 3)];
            gst(a.partb, (long)blockIdx.x * a.co + cb * 16 + k, sacc);
        }
    }
}

// dW[co][tap][ci] (the flat parameter layout) and db[co] from the partials,
// summed over chunks in a fixed order: first per group of consecutive
// chunks (one thread per output and group), then over the groups in order
constexpr int kRedGroups = 64;

__global__ void k_wgrad_reduce1(const float *__restrict__ part, const float *__restrict__ partb, int nch, int ngrp, int ci,
                                int co, float *__restrict__ red) {
    const int nout = ci * co, tot = 27 * nout + co;
    const int q = blockIdx.x * blockDim.x + threadIdx.x, g = blockIdx.y;
    if (q >= tot) return;
    const int c0 = (int)((long)nch * g / ngrp), c1 = (int)((long)nch * (g + 1) / ngrp);
    float s = 0.0f;
    if (q < 27 * nout) {
        for (int c = c0; c < c1; c++) s += gld(part, (long)c * 27 * nout + q);
    } else {
        for (int c = c0; c < c1; c++) s += gld(partb, (long)c * co + (q - 27 * nout));
    }
    gst(red, (long)g * tot + q, s);
}

__global__ void k_wgrad_reduce2(const float *__restrict__ red, int ngrp, int ci, int co, float *__restrict__ dw,
                                float *__restrict__ db) {
    const int nout = ci * co, tot = 27 * nout + co;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= tot) return;
    float s = 0.0f;
    for (int g = 0; g < ngrp; g++) s += gld(red, (long)g * tot + q);
    if (q < 27 * nout) {
        const int tap = q / nout, o = q % nout, oc = o / ci, ic = o % ci;
        gst(dw, ((long)oc * 27 + tap) * ci + ic, s);
    } else {
        gst(db, q - 27 * nout, s);
    }
}

// ---------------------------------------------------------- elementwise
// 8 bf16 <-> 8 floats
__device__ __forceinline__ void unpack8(const u32x4 v, float *f) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
        f[2 * i] = __uint_as_float(v[i] << 16);
        f[2 * i + 1] = __uint_as_float(v[i] & 0xFFFF0000u);
    }
}
__device__ __forceinline__ u32x4 pack8(const float *f) {
    return u32x4{f2bf2_hw(f[0], f[1]), f2bf2_hw(f[2], f[3]), f2bf2_hw(f[4], f[5]), f2bf2_hw(f[6], f[7])};
}

// mean of the 2x2x2 children, rounded to bf16; one thread per coarse cell
// and group of 8 channels
__global__ void k_pool(const u16 *__restrict__ in, u16 *__restrict__ out, int nx, int ny, int nz, int cs) {
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2, ng = cs >> 3;
    const long n = (long)cx * cy * cz * ng;
    const u32x4 *src = (const u32x4 *)in;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int gq = (int)(q % ng);
        const long v = q / ng;
        const int I = (int)(v % cx), J = (int)((v / cx) % cy), K = (int)(v / ((long)cx * cy));
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < 2; kk++)
            for (int jj = 0; jj < 2; jj++)
                for (int ii = 0; ii < 2; ii++) {
                    float f[8];
                    unpack8(gld(src, ((2 * I + ii) + nx * ((2 * J + jj) + (long)ny * (2 * K + kk))) * ng + gq), f);
#pragma unroll
                    for (int c = 0; c < 8; c++) s[c] += f[c];
                }
#pragma unroll
        for (int c = 0; c < 8; c++) s[c] *= 0.125f;
        gst((u32x4 *)out, q, pack8(s));
    }
}

// s = upsample(t) + e (nearest), rounded to bf16; one thread per cell and
// group of 8 channels
__global__ void k_upadd(const u16 *__restrict__ t, const u16 *__restrict__ e, u16 *__restrict__ s, int nx, int ny, int nz,
                        int cs) {
    const int ng = cs >> 3;
    const long n = (long)nx * ny * nz * ng;
    const int cx = nx / 2, cy = ny / 2;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int gq = (int)(q % ng);
        const long v = q / ng;
        const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((long)nx * ny));
        const long pv = (i / 2) + cx * ((j / 2) + (long)cy * (k / 2));
        float a[8], b[8];
        unpack8(gld((const u32x4 *)t, pv * ng + gq), a);
        unpack8(gld((const u32x4 *)e, q), b);
#pragma unroll
        for (int c = 0; c < 8; c++) a[c] += b[c];
        gst((u32x4 *)s, q, pack8(a));
    }
}

// g *= (act > 0)
__global__ void k_relu_bwd(float *__restrict__ g, const u16 *__restrict__ act, long n) {
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x)
        if (!(bf2f(gld(act, q)) > 0.0f)) gst(g, q, 0.0f);
}

// adjoint of nearest upsampling: coarse gradient = sum of the 8 children
__global__ void k_up_bwd(const float *__restrict__ gs, float *__restrict__ gt, int nx, int ny, int nz, int cs) {
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const long n = (long)cx * cy * cz * cs;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int c = (int)(q % cs);
        const long v = q / cs;
        const int I = (int)(v % cx), J = (int)((v / cx) % cy), K = (int)(v / ((long)cx * cy));
        float s = 0.0f;
        for (int kk = 0; kk < 2; kk++)
            for (int jj = 0; jj < 2; jj++)
                for (int ii = 0; ii < 2; ii++)
                    s += gld(gs, ((2 * I + ii) + nx * ((2 * J + jj) + (long)ny * (2 * K + kk))) * cs + c);
        gst(gt, q, s);
    }
}

// fine gradient = (adjoint of the 2x2x2 mean: coarse gradient / 8) + skip
__global__ void k_pool_bwd_add(const float *__restrict__ gp, const float *__restrict__ skip, float *__restrict__ g, int nx,
                               int ny, int nz, int cs) {
    const long n = (long)nx * ny * nz * cs;
    const int cx = nx / 2, cy = ny / 2;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int c = (int)(q % cs);
        const long v = q / cs;
        const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((long)nx * ny));
        const long pv = (i / 2) + cx * ((j / 2) + (long)cy * (k / 2));
        gst(g, q, gld(gp, pv * cs + c) * 0.125f + gld(skip, q));
    }
}

// [cell][cin] bf16 -> [cell][cs] bf16 with zero channels; one thread per
// cell and group of 8 channels
__global__ void k_in_pad(const u16 *__restrict__ in, int cin, u16 *__restrict__ out, int cs, long ncell) {
    const int ng = cs >> 3;
    const long n = ncell * ng;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int gq = (int)(q % ng);
        const long v = q / ng;
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const int cc = gq * 8 + c;
            const uint32_t h = cc < cin ? (uint32_t)gld(in, v * cin + cc) : 0u;
            w[c >> 1] |= h << (16 * (c & 1));
        }
        gst((u32x4 *)out, q, u32x4{w[0], w[1], w[2], w[3]});
    }
}

// mean squared error: gradient 2 (out - target) / n into channel 0 of a
// [cell][cs] buffer, per-block partial sums of the squares
__global__ void __launch_bounds__(256) k_mse(const float *__restrict__ out, const float *__restrict__ target, long n, int cs,
                                             float *__restrict__ g, double *__restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const float d = gld(out, q) - gld(target, q);
        s += (double)d * d;
        gst(g, q * cs, 2.0f * d / (float)n);
        for (int c = 1; c < cs; c++) gst(g, q * cs + c, 0.0f);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) gst(part, (long)blockIdx.x, s);
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v, long n,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const float gq = gld(g, q);
        const float mq = b1 * gld(m, q) + (1.0f - b1) * gq;
        const float vq = b2 * gld(v, q) + (1.0f - b2) * gq * gq;
        gst(m, q, mq);
        gst(v, q, vq);
        gst(p, q, gld(p, q) - lr * (mq / c1) / (sqrtf(vq / c2) + eps));
    }
}

// network input of the warm start: channel 0 = rho * scale0, channel 1 the
// electrode ramp ramp0 + ramp1 * (i + 1/2)
__global__ void k_features(const double *__restrict__ rho, long ncell, int nx, double scale0, double ramp0, double ramp1,
                           u16 *__restrict__ out) {
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < ncell; q += (long)gridDim.x * blockDim.x) {
        const int i = (int)(q % nx);
        gst(out, 2 * q, f2bf((float)(gld(rho, q) * scale0)));
        gst(out, 2 * q + 1, f2bf((float)(ramp0 + ramp1 * (i + 0.5))));
    }
}

__global__ void k_guess_to_x(const float *__restrict__ out, double vref, double *__restrict__ x, long n) {
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x)
        gst(x, q, vref * (double)gld(out, q));
}

// ------------------------------------------------------------ host side
static int pow2pad(int c) {
    int p = 8;
    while (p < c) p *= 2;
    return p;
}
static int lg2(int p) {
    int l = 0;
    while ((1 << l) < p) l++;
    return l;
}
static int grid_for(long n) { return (int)std::min<long>((n + 255) / 256, 8192); }

// cell blocks per weight-gradient chunk: enough workgroups to fill the
// chip (>= 2048 with the block pairs), at most 16 blocks per chunk
static int wgrad_tpc(int ntiles, int pairs) {
    int tpc = 16;
    while (tpc > 1 && (long)((ntiles + tpc - 1) / tpc) * pairs < 2048) tpc /= 2;
    return tpc;
}
static int conv_tiles(int nx, int ny, int nz) {
    return ((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY) * ((nz + kTZ - 1) / kTZ);
}
// weight-gradient chunks of a ci -> co convolution on an nx x ny x nz grid
static int wgrad_chunks(int ci, int co, int nx, int ny, int nz) {
    const int nt = conv_tiles(nx, ny, nz), pairs = ((co + 15) / 16) * ((ci + 15) / 16);
    const int tpc = wgrad_tpc(nt, pairs);
    return (nt + tpc - 1) / tpc;
}


struct Conv {
    int ci, co, cis, cos, nch, cop, nchT, cipT;
    long woff, boff;
    DevBuf<u16> wf, wt;
    void init(int ci_, int co_) {
        ci = ci_; co = co_;
        cis = pow2pad(ci); cos = pow2pad(co);
        nch = (cis + 15) / 16;
        cop = std::max((co + 15) / 16 * 16, cos);
        nchT = (cos + 15) / 16;
        cipT = std::max((ci + 15) / 16 * 16, cis);
        wf.alloc((size_t)cop * nch * 448);
        wt.alloc((size_t)cipT * nchT * 448);
    }
    void pack(const float *w, hipStream_t s) {
        k_pack<<<grid_for((long)cop * nch * 448 + (long)cipT * nchT * 448), 256, 0, s>>>(w, ci, co, nch, cop, wf.p, nchT, cipT,
                                                                                         wt.p);
    }
};

struct Level {
    int nx = 0, ny = 0, nz = 0;
    long n = 0;
    DevBuf<u16> in, a, e, t, s, d;     // t: t_{l-1} (level l holds the up-conv output of level l-1)
    DevBuf<float> g1, g2, gs;
};

struct Net {
    vd_nn_config cfg;
    std::vector<Conv> convs;
    std::vector<int> enc_a, enc_b, up, dec;
    int out_conv = -1;
    long nparam = 0;
    DevBuf<float> params, grads, m, v;
    long step = 0;
    bool packed = false;
    int gx = 0, gy = 0, gz = 0;          // grid the activations are sized for
    std::vector<Level> lv;
    DevBuf<float> out, gout;
    DevBuf<float> part, partb, red;
    DevBuf<double> mse_part;
    double *pin_loss = nullptr;
    DevBuf<u16> feat;
    ~Net() { if (pin_loss) (void)hipHostFree(pin_loss); }
};

static long conv_count(const vd_nn_config &c, std::vector<std::pair<int, int>> *shapes) {
    long n = 0;
    auto add = [&](int ci, int co) {
        if (shapes) shapes->push_back({ci, co});
        n += (long)co * 27 * ci + co;
    };
    for (int l = 0; l < c.levels; l++) {
        add(l == 0 ? c.cin : c.ch[l - 1], c.ch[l]);
        add(c.ch[l], c.ch[l]);
    }
    for (int l = c.levels - 2; l >= 0; l--) {
        add(c.ch[l + 1], c.ch[l]);
        add(c.ch[l], c.ch[l]);
    }
    add(c.ch[0], 1);
    return n;
}

static void check_cfg(const vd_nn_config *c) {
    VD_CHECK(c, "null config");
    VD_CHECK(c->levels >= 1 && c->levels <= 4, "levels must be 1..4");
    VD_CHECK(c->cin >= 1 && c->cin <= 8, "cin must be 1..8");
    for (int l = 0; l < c->levels; l++) VD_CHECK(c->ch[l] >= 1 && c->ch[l] <= 64, "channels must be 1..64");
}

static Net &net_of(vd_ctx *ctx) {
    auto it = ctx->cache.find("nn:net");
    VD_CHECK(it != ctx->cache.end(), "no network: call vd_nn_create first");
    return *std::static_pointer_cast<Net>(it->second);
}

static void size_for_grid(vd_ctx *ctx, Net &N, int nx, int ny, int nz) {
    const int L = N.cfg.levels;
    VD_CHECK(nx > 0 && ny > 0 && nz > 0, "grid must be positive");
    VD_CHECK(nx % (1 << (L - 1)) == 0 && ny % (1 << (L - 1)) == 0 && nz % (1 << (L - 1)) == 0,
             "grid must be divisible by 2^(levels-1)");
    if (N.gx == nx && N.gy == ny && N.gz == nz) return;
    VD_HIP(hipStreamSynchronize(ctx->stream));
    N.lv.clear();
    N.lv.resize(L);
    const int *ch = N.cfg.ch;
    for (int l = 0; l < L; l++) {
        Level &V = N.lv[l];
        V.nx = nx >> l; V.ny = ny >> l; V.nz = nz >> l;
        V.n = (long)V.nx * V.ny * V.nz;
        const int cs = pow2pad(ch[l]);
        const int cprev = l > 0 ? pow2pad(ch[l - 1]) : pow2pad(N.cfg.cin);
        V.in.alloc((size_t)V.n * cprev);
        V.a.alloc((size_t)V.n * cs);
        V.e.alloc((size_t)V.n * cs);
        if (l > 0) V.t.alloc((size_t)V.n * cprev);
        if (l < L - 1) { V.s.alloc((size_t)V.n * cs); V.d.alloc((size_t)V.n * cs); }
        const int gcap = std::max(cs, cprev);
        V.g1.alloc((size_t)V.n * gcap);
        V.g2.alloc((size_t)V.n * gcap);
        V.gs.alloc((size_t)V.n * cs);
    }
    if (L == 1) N.lv[0].d.alloc((size_t)N.lv[0].n * pow2pad(ch[0]));
    const long n0 = N.lv[0].n;
    N.out.alloc(n0);
    N.gout.alloc((size_t)n0 * 8);
    N.feat.alloc((size_t)n0 * 2);
    // gradient partials: the largest need over the convolutions, each at
    // the level it runs on (the up-convolution of level l on level l + 1)
    long pmax = 0, pbmax = 0;
    auto need = [&](int idx, int l) {
        const Conv &c = N.convs[idx];
        const Level &V = N.lv[l];
        const long nc = wgrad_chunks(c.ci, c.co, V.nx, V.ny, V.nz);
        pmax = std::max(pmax, nc * 27 * c.ci * c.co);
        pbmax = std::max(pbmax, nc * c.co);
    };
    for (int l = 0; l < L; l++) { need(N.enc_a[l], l); need(N.enc_b[l], l); }
    for (int l = L - 2; l >= 0; l--) { need(N.up[l], l + 1); need(N.dec[l], l); }
    need(N.out_conv, 0);
    N.part.alloc((size_t)pmax);
    N.partb.alloc((size_t)pbmax);
    long rmax = 0;
    for (auto &c : N.convs) rmax = std::max(rmax, (long)kRedGroups * (27L * c.ci * c.co + c.co));
    N.red.alloc((size_t)rmax);
    N.mse_part.alloc(grid_for(n0));
    N.gx = nx; N.gy = ny; N.gz = nz;
}

static void pack_all(vd_ctx *ctx, Net &N) {
    for (auto &c : N.convs) c.pack(N.params.p + c.woff, ctx->stream);
    VD_HIP(hipGetLastError());
    N.packed = true;
}

// one convolution; transposed = input-gradient form (in: FP32 gradient with
// cos channels, out: FP32 with cis channels)
static void run_conv(vd_ctx *ctx, Net &N, const Conv &c, const Level &V, const void *in, bool in_f32, void *out, bool out_f32,
                     int out_s, bool relu, bool transposed) {
    ConvArgs a;
    a.in = in;
    a.cin_s = transposed ? c.cos : c.cis;
    a.nx = V.nx; a.ny = V.ny; a.nz = V.nz;
    a.w = transposed ? c.wt.p : c.wf.p;
    a.bias = transposed ? nullptr : N.params.p + c.boff;
    a.out = out; a.out_f32 = out_f32 ? 1 : 0; a.out_s = out_s;
    a.co = transposed ? c.ci : c.co;
    a.relu = relu ? 1 : 0;
    const int cop = transposed ? c.cipT : c.cop;
    const int ncb = cop / 16;                      // 16-column blocks
    const long nblk = (long)((V.nx + kTX - 1) / kTX) * ((V.ny + kTY - 1) / kTY) * ((V.nz + kTZ - 1) / kTZ);
    VD_CHECK(ncb >= 1 && ncb <= 4 && cop % 16 == 0, "internal: conv width");
    VD_CHECK(out_s <= cop, "internal: conv output stride");
    VD_CHECK(nblk <= 0x7fffffffL, "internal: conv grid");
    VD_CHECK(V.n * std::max(a.cin_s, out_s) < (1L << 31), "grid too large for the convolution kernels");
    // two column blocks per workgroup where that still leaves >= 4096
    // workgroups, else one (coarse levels: more workgroups, each restaging
    // the same input block)
    const int nb = (ncb % 2 == 0 && nblk * (ncb / 2) >= 4096) ? 2 : 1;
    // inputs of one 16-channel chunk march along z (kZS slabs per workgroup)
    const long nblk_z = (long)((V.nx + kTX - 1) / kTX) * ((V.ny + kTY - 1) / kTY) * ((V.nz + 2 * kZS - 1) / (2 * kZS));
    const bool march = a.cin_s <= 16 && nblk_z * (ncb / nb) >= 1024;
    const dim3 grid((unsigned)(march ? nblk_z : nblk), (unsigned)(ncb / nb));
    timed(ctx, "nn_conv", 0.0, [&] {
#define VD_CONV(K_, NB_)                                                                  \
    if (in_f32) K_<NB_, true><<<grid, 64 * kConvWaves, 0, ctx->stream>>>(a);            \
    else K_<NB_, false><<<grid, 64 * kConvWaves, 0, ctx->stream>>>(a);
        if (march) {
            if (nb == 2) { VD_CONV(k_conv_z, 2) }
            else { VD_CONV(k_conv_z, 1) }
        } else {
            if (nb == 2) { VD_CONV(k_conv, 2) }
            else { VD_CONV(k_conv, 1) }
        }
#undef VD_CONV
    });
}

static void run_wgrad(vd_ctx *ctx, Net &N, const Conv &c, const Level &V, const u16 *x, const float *dy) {
    WgArgs a;
    a.x = x; a.xs = c.cis; a.ci = c.ci;
    a.dy = dy; a.dys = c.cos; a.co = c.co;
    a.nx = V.nx; a.ny = V.ny; a.nz = V.nz;
    const int ntiles = conv_tiles(V.nx, V.ny, V.nz);
    const int pairs = ((c.co + 15) / 16) * ((c.ci + 15) / 16);
    a.tiles_per_chunk = wgrad_tpc(ntiles, pairs);
    const int nch = (ntiles + a.tiles_per_chunk - 1) / a.tiles_per_chunk;
    VD_CHECK(nch == wgrad_chunks(c.ci, c.co, V.nx, V.ny, V.nz), "internal: gradient chunks");
    VD_CHECK((size_t)nch * 27 * c.ci * c.co <= N.part.n && (size_t)nch * c.co <= N.partb.n, "internal: gradient partials");
    a.part = N.part.p; a.partb = N.partb.p;
    const int tot = 27 * c.ci * c.co + c.co;
    const int ngrp = std::min(kRedGroups, nch);
    VD_CHECK((size_t)ngrp * tot <= N.red.n, "internal: gradient reduction buffer");
    timed(ctx, "nn_wgrad", 0.0, [&] {
        k_wgrad<<<dim3(nch, pairs), 256, 0, ctx->stream>>>(a);
        k_wgrad_reduce1<<<dim3((tot + 255) / 256, ngrp), 256, 0, ctx->stream>>>(N.part.p, N.partb.p, nch, ngrp, c.ci, c.co,
                                                                                N.red.p);
        k_wgrad_reduce2<<<(tot + 255) / 256, 256, 0, ctx->stream>>>(N.red.p, ngrp, c.ci, c.co, N.grads.p + c.woff,
                                                                   N.grads.p + c.boff);
    });
}

static void forward(vd_ctx *ctx, Net &N, const u16 *in_cin) {
    if (!N.packed) pack_all(ctx, N);
    const int L = N.cfg.levels;
    hipStream_t s = ctx->stream;
    Level &V0 = N.lv[0];
    const int cin_s = pow2pad(N.cfg.cin);
    k_in_pad<<<grid_for(V0.n * cin_s / 8), 256, 0, s>>>(in_cin, N.cfg.cin, V0.in.p, cin_s, V0.n);
    for (int l = 0; l < L; l++) {
        Level &V = N.lv[l];
        const Conv &ca = N.convs[N.enc_a[l]], &cb = N.convs[N.enc_b[l]];
        if (l > 0) {
            const Level &P = N.lv[l - 1];
            k_pool<<<grid_for(V.n * ca.cis / 8), 256, 0, s>>>(P.e.p, V.in.p, P.nx, P.ny, P.nz, ca.cis);
        }
        run_conv(ctx, N, ca, V, V.in.p, false, V.a.p, false, ca.cos, true, false);
        run_conv(ctx, N, cb, V, V.a.p, false, V.e.p, false, cb.cos, true, false);
    }
    const u16 *d = N.lv[L - 1].e.p;
    for (int l = L - 2; l >= 0; l--) {
        Level &V = N.lv[l], &C = N.lv[l + 1];
        const Conv &cu = N.convs[N.up[l]], &cd = N.convs[N.dec[l]];
        run_conv(ctx, N, cu, C, d, false, C.t.p, false, cu.cos, true, false);
        k_upadd<<<grid_for(V.n * cu.cos / 8), 256, 0, s>>>(C.t.p, V.e.p, V.s.p, V.nx, V.ny, V.nz, cu.cos);
        run_conv(ctx, N, cd, V, V.s.p, false, V.d.p, false, cd.cos, true, false);
        d = V.d.p;
    }
    const Conv &co = N.convs[N.out_conv];
    run_conv(ctx, N, co, V0, d, false, N.out.p, true, 1, false, false);
    VD_HIP(hipGetLastError());
}

// gradient of the loss with respect to every parameter (N.gout holds the
// output gradient, channel 0 of a stride-8 buffer)
static void backward(vd_ctx *ctx, Net &N) {
    const int L = N.cfg.levels;
    hipStream_t s = ctx->stream;
    auto d_of = [&](int l) -> const u16 * { return l == L - 1 ? N.lv[L - 1].e.p : N.lv[l].d.p; };
    Level &V0 = N.lv[0];
    const Conv &co = N.convs[N.out_conv];
    run_wgrad(ctx, N, co, V0, d_of(0), N.gout.p);
    run_conv(ctx, N, co, V0, N.gout.p, true, V0.g1.p, true, co.cis, false, true);   // g_d0
    for (int l = 0; l <= L - 2; l++) {
        Level &V = N.lv[l], &C = N.lv[l + 1];
        const Conv &cd = N.convs[N.dec[l]], &cu = N.convs[N.up[l]];
        k_relu_bwd<<<grid_for(V.n * cd.cos), 256, 0, s>>>(V.g1.p, V.d.p, V.n * cd.cos);
        run_wgrad(ctx, N, cd, V, V.s.p, V.g1.p);
        run_conv(ctx, N, cd, V, V.g1.p, true, V.gs.p, true, cd.cis, false, true);    // g_s
        k_up_bwd<<<grid_for(C.n * cu.cos), 256, 0, s>>>(V.gs.p, C.g2.p, V.nx, V.ny, V.nz, cu.cos);
        k_relu_bwd<<<grid_for(C.n * cu.cos), 256, 0, s>>>(C.g2.p, C.t.p, C.n * cu.cos);
        run_wgrad(ctx, N, cu, C, d_of(l + 1), C.g2.p);
        run_conv(ctx, N, cu, C, C.g2.p, true, C.g1.p, true, cu.cis, false, true);    // g_d_{l+1}
    }
    for (int l = L - 1; l >= 0; l--) {
        Level &V = N.lv[l];
        const Conv &ca = N.convs[N.enc_a[l]], &cb = N.convs[N.enc_b[l]];
        if (l < L - 1) {
            const Level &C = N.lv[l + 1];
            (void)C;
            k_pool_bwd_add<<<grid_for(V.n * cb.cos), 256, 0, s>>>(N.lv[l + 1].g1.p, V.gs.p, V.g1.p, V.nx, V.ny, V.nz, cb.cos);
        }
        k_relu_bwd<<<grid_for(V.n * cb.cos), 256, 0, s>>>(V.g1.p, V.e.p, V.n * cb.cos);
        run_wgrad(ctx, N, cb, V, V.a.p, V.g1.p);
        run_conv(ctx, N, cb, V, V.g1.p, true, V.g2.p, true, cb.cis, false, true);     // g_a
        k_relu_bwd<<<grid_for(V.n * ca.cos), 256, 0, s>>>(V.g2.p, V.a.p, V.n * ca.cos);
        run_wgrad(ctx, N, ca, V, V.in.p, V.g2.p);
        if (l > 0) run_conv(ctx, N, ca, V, V.g2.p, true, V.g1.p, true, ca.cis, false, true);   // g_p
    }
    VD_HIP(hipGetLastError());
}

}  // namespace nn

// ------------------------------------------------------------ entry points
vd_status nn_create(vd_ctx *ctx, const vd_nn_config *cfg, const float *params) {
    using namespace nn;
    check_cfg(cfg);
    auto N = std::make_shared<Net>();
    N->cfg = *cfg;
    std::vector<std::pair<int, int>> shapes;
    N->nparam = conv_count(*cfg, &shapes);
    long off = 0;
    for (auto &sh : shapes) {
        Conv c;
        c.init(sh.first, sh.second);
        c.woff = off;
        off += (long)c.co * 27 * c.ci;
        c.boff = off;
        off += c.co;
        N->convs.push_back(std::move(c));
    }
    int q = 0;
    for (int l = 0; l < cfg->levels; l++) { N->enc_a.push_back(q++); N->enc_b.push_back(q++); }
    N->up.assign(cfg->levels, -1);
    N->dec.assign(cfg->levels, -1);
    for (int l = cfg->levels - 2; l >= 0; l--) { N->up[l] = q++; N->dec[l] = q++; }
    N->out_conv = q++;
    N->params.alloc(N->nparam);
    N->grads.alloc(N->nparam);
    N->m.alloc(N->nparam);
    N->v.alloc(N->nparam);
    if (params) VD_HIP(hipMemcpyAsync(N->params.p, params, sizeof(float) * N->nparam, hipMemcpyHostToDevice, ctx->stream));
    else VD_HIP(hipMemsetAsync(N->params.p, 0, sizeof(float) * N->nparam, ctx->stream));
    VD_HIP(hipMemsetAsync(N->m.p, 0, sizeof(float) * N->nparam, ctx->stream));
    VD_HIP(hipMemsetAsync(N->v.p, 0, sizeof(float) * N->nparam, ctx->stream));
    VD_HIP(hipMemsetAsync(N->grads.p, 0, sizeof(float) * N->nparam, ctx->stream));
    VD_HIP(hipHostMalloc((void **)&N->pin_loss, sizeof(double), hipHostMallocDefault));
    VD_HIP(hipStreamSynchronize(ctx->stream));
    ctx->cache["nn:net"] = N;
    return VD_OK;
}

int64_t nn_param_count(const vd_nn_config *cfg) {
    nn::check_cfg(cfg);
    return nn::conv_count(*cfg, nullptr);
}

vd_status nn_params(vd_ctx *ctx, int which, float *host, int set) {
    nn::Net &N = nn::net_of(ctx);
    VD_CHECK(host, "null buffer");
    VD_CHECK(which >= 0 && which <= 3, "which must be 0 (params), 1 (grads), 2 (m), 3 (v)");
    float *d = which == 0 ? N.params.p : which == 1 ? N.grads.p : which == 2 ? N.m.p : N.v.p;
    if (set) {
        VD_HIP(hipMemcpyAsync(d, host, sizeof(float) * N.nparam, hipMemcpyHostToDevice, ctx->stream));
        if (which == 0) N.packed = false;
    } else {
        VD_HIP(hipMemcpyAsync(host, d, sizeof(float) * N.nparam, hipMemcpyDeviceToHost, ctx->stream));
    }
    VD_HIP(hipStreamSynchronize(ctx->stream));
    return VD_OK;
}

vd_status nn_forward(vd_ctx *ctx, const vd_grid *g, const uint16_t *in, float *out) {
    nn::Net &N = nn::net_of(ctx);
    VD_CHECK(g && in && out, "null argument");
    nn::size_for_grid(ctx, N, g->nx, g->ny, g->nz);
    nn::forward(ctx, N, in);
    VD_HIP(hipMemcpyAsync(out, N.out.p, sizeof(float) * N.lv[0].n, hipMemcpyDeviceToDevice, ctx->stream));
    return VD_OK;
}

vd_status nn_train_step(vd_ctx *ctx, const vd_grid *g, const uint16_t *in, const float *target, float lr, int update,
                        double *loss) {
    using namespace nn;
    Net &N = net_of(ctx);
    VD_CHECK(g && in && target, "null argument");
    VD_CHECK(lr >= 0.0f, "learning rate must be >= 0");
    size_for_grid(ctx, N, g->nx, g->ny, g->nz);
    forward(ctx, N, in);
    const long n0 = N.lv[0].n;
    const int nb = grid_for(n0);
    k_mse<<<nb, 256, 0, ctx->stream>>>(N.out.p, target, n0, 8, N.gout.p, N.mse_part.p);
    backward(ctx, N);
    if (update) {
        N.step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - powf(b1, (float)N.step), c2 = 1.0f - powf(b2, (float)N.step);
        k_adam<<<grid_for(N.nparam), 256, 0, ctx->stream>>>(N.params.p, N.grads.p, N.m.p, N.v.p, N.nparam, lr, b1, b2, 1e-8f,
                                                            c1, c2);
        N.packed = false;
        pack_all(ctx, N);
    }
    VD_HIP(hipGetLastError());
    if (loss) {
        std::vector<double> part(nb);
        VD_HIP(hipMemcpyAsync(part.data(), N.mse_part.p, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
        VD_HIP(hipStreamSynchronize(ctx->stream));
        double s = 0.0;
        for (double v : part) s += v;
        *loss = s / (double)n0;
    }
    return VD_OK;
}

// scale of the network input and output for a potential problem: channel 0
// = rho Lx^2 / (eps V), channel 1 = electrode ramp / V along x (the Laplace
// solution between two plates with zero-flux side walls), V the largest
// |Dirichlet value| (1 if none is non-zero)
static void feature_scale(const vd_grid *g, const vd_bc *bc, double eps, double *vref, double *s0, double *r0, double *r1) {
    double V = 0.0;
    for (int f = 0; f < 6; f++)
        if (bc->kind[f] == VD_BC_DIRICHLET) V = std::max(V, std::fabs(bc->value[f]));
    if (V == 0.0) V = 1.0;
    const double Lx = g->nx * g->dx;
    *vref = V;
    *s0 = Lx * Lx / (eps * V);
    if (bc->kind[0] == VD_BC_DIRICHLET && bc->kind[1] == VD_BC_DIRICHLET) {
        *r0 = bc->value[0] / V;
        *r1 = (bc->value[1] - bc->value[0]) / V / g->nx;
    } else {
        *r0 = 0.0;
        *r1 = 0.0;
    }
}

vd_status nn_features(vd_ctx *ctx, const vd_grid *g, const vd_bc *bc, const double *rho, double eps, uint16_t *out,
                      double *vref) {
    VD_CHECK(g && bc && rho && out && eps > 0.0, "bad argument");
    double V, s0, r0, r1;
    feature_scale(g, bc, eps, &V, &s0, &r0, &r1);
    const long n = (long)g->nx * g->ny * g->nz;
    nn::k_features<<<nn::grid_for(n), 256, 0, ctx->stream>>>(rho, n, g->nx, s0, r0, r1, out);
    VD_HIP(hipGetLastError());
    if (vref) *vref = V;
    return VD_OK;
}

// the learned guess written into x (FP64): x = V * net(features(rho))
vd_status nn_guess(vd_ctx *ctx, const vd_grid *g, const vd_bc *bc, const double *rho, double eps, double *x) {
    nn::Net &N = nn::net_of(ctx);
    VD_CHECK(N.cfg.cin == 2, "the warm-start network takes 2 input channels");
    nn::size_for_grid(ctx, N, g->nx, g->ny, g->nz);
    double V;
    nn_features(ctx, g, bc, rho, eps, N.feat.p, &V);
    nn::forward(ctx, N, N.feat.p);
    const long n = N.lv[0].n;
    nn::k_guess_to_x<<<nn::grid_for(n), 256, 0, ctx->stream>>>(N.out.p, V, x, n);
    VD_HIP(hipGetLastError());
    return VD_OK;
}

// network file: 8-byte tag, the configuration, the parameter count, then
// the FP32 parameters (little-endian, the flat order of the parameters)
static const char kNnTag[8] = {'V', 'D', 'N', 'N', '0', '0', '0', '1'};

vd_status nn_save(vd_ctx *ctx, const char *path) {
    nn::Net &N = nn::net_of(ctx);
    VD_CHECK(path, "null path");
    std::vector<float> h(N.nparam);
    nn_params(ctx, 0, h.data(), 0);
    FILE *f = fopen(path, "wb");
    VD_CHECK(f, std::string("cannot open ") + path);
    const int64_t np = N.nparam;
    bool ok = fwrite(kNnTag, 1, 8, f) == 8 && fwrite(&N.cfg, sizeof(N.cfg), 1, f) == 1 && fwrite(&np, sizeof(np), 1, f) == 1 &&
              fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    ok = (fclose(f) == 0) && ok;
    VD_CHECK(ok, std::string("write failed: ") + path);
    return VD_OK;
}

vd_status nn_load(vd_ctx *ctx, const char *path) {
    VD_CHECK(path, "null path");
    FILE *f = fopen(path, "rb");
    VD_CHECK(f, std::string("cannot open ") + path);
    char tag[8];
    vd_nn_config cfg;
    int64_t np = 0;
    bool ok = fread(tag, 1, 8, f) == 8 && memcmp(tag, kNnTag, 8) == 0 && fread(&cfg, sizeof(cfg), 1, f) == 1 &&
              fread(&np, sizeof(np), 1, f) == 1;
    std::vector<float> h;
    if (ok) {
        try { ok = np == nn_param_count(&cfg); } catch (...) { ok = false; }
    }
    if (ok) {
        h.resize(np);
        ok = fread(h.data(), sizeof(float), h.size(), f) == h.size();
    }
    fclose(f);
    VD_CHECK(ok, std::string("not a network file of this library: ") + path);
    return nn_create(ctx, &cfg, h.data());
}

// layer-level entry points (one convolution and its gradients)
vd_status nn_conv3d(vd_ctx *ctx, const vd_grid *g, const uint16_t *x, int ci, const float *w, const float *b, int co, int relu,
                    float *y, const float *dy, float *dx, float *dw, float *db) {
    using namespace nn;
    VD_CHECK(g && x && w && ci >= 1 && ci <= 64 && co >= 1 && co <= 64, "bad argument");
    const long n = (long)g->nx * g->ny * g->nz;
    VD_CHECK(n > 0, "empty grid");
    Net N;
    N.cfg.levels = 1;
    N.nparam = (long)co * 27 * ci + co;
    Conv c;
    c.init(ci, co);
    c.woff = 0;
    c.boff = (long)co * 27 * ci;
    N.params.alloc(N.nparam);
    N.grads.alloc(N.nparam);
    hipStream_t s = ctx->stream;
    VD_HIP(hipMemcpyAsync(N.params.p, w, sizeof(float) * c.boff, hipMemcpyDeviceToDevice, s));
    if (b) VD_HIP(hipMemcpyAsync(N.params.p + c.boff, b, sizeof(float) * co, hipMemcpyDeviceToDevice, s));
    else VD_HIP(hipMemsetAsync(N.params.p + c.boff, 0, sizeof(float) * co, s));
    c.pack(N.params.p, s);
    Level V;
    V.nx = g->nx; V.ny = g->ny; V.nz = g->nz; V.n = n;
    DevBuf<u16> xin;
    xin.alloc((size_t)n * c.cis);
    k_in_pad<<<grid_for(n * c.cis / 8), 256, 0, s>>>(x, ci, xin.p, c.cis, n);
    DevBuf<float> tmp;
    tmp.alloc((size_t)n * std::max(c.cos, c.cis));
    if (y) {
        run_conv(ctx, N, c, V, xin.p, false, tmp.p, true, c.cos, relu != 0, false);
        VD_HIP(hipMemcpy2DAsync(y, sizeof(float) * co, tmp.p, sizeof(float) * c.cos, sizeof(float) * co, n,
                                hipMemcpyDeviceToDevice, s));
    }
    if (dy) {
        VD_CHECK(dx && dw && db, "the backward needs dx, dw and db");
        DevBuf<float> dyp;
        dyp.alloc((size_t)n * c.cos);
        VD_HIP(hipMemsetAsync(dyp.p, 0, sizeof(float) * n * c.cos, s));
        VD_HIP(hipMemcpy2DAsync(dyp.p, sizeof(float) * c.cos, dy, sizeof(float) * co, sizeof(float) * co, n,
                                hipMemcpyDeviceToDevice, s));
        const long nch = wgrad_chunks(ci, co, g->nx, g->ny, g->nz);
        N.part.alloc((size_t)nch * 27 * ci * co);
        N.partb.alloc((size_t)nch * co);
        N.red.alloc((size_t)kRedGroups * (27L * ci * co + co));
        run_wgrad(ctx, N, c, V, xin.p, dyp.p);
        run_conv(ctx, N, c, V, dyp.p, true, tmp.p, true, c.cis, false, true);
        VD_HIP(hipMemcpy2DAsync(dx, sizeof(float) * ci, tmp.p, sizeof(float) * c.cis, sizeof(float) * ci, n,
                                hipMemcpyDeviceToDevice, s));
        VD_HIP(hipMemcpyAsync(dw, N.grads.p, sizeof(float) * c.boff, hipMemcpyDeviceToDevice, s));
        VD_HIP(hipMemcpyAsync(db, N.grads.p + c.boff, sizeof(float) * co, hipMemcpyDeviceToDevice, s));
    }
    VD_HIP(hipGetLastError());
    VD_HIP(hipStreamSynchronize(s));
    return VD_OK;
}

}  // namespace vd
