// Learned initial guess for the Poisson solve (Sec. 2.1, Eqs. (3)-(4);
// multigrid of Sec. 4): a small 3D U-Net maps the scaled charge density and
// the electrode ramp to the scaled potential.  Not part of the paper's
// method; the multigrid solve that follows still decides convergence.
//
// Layout: activations are channels-last, [cell][channel] with the channel
// stride padded to a power of two >= 8, stored as bfloat16; gradients are
// FP32 in the same layout.  A 3x3x3 convolution is an implicit GEMM
// (M = cells, N = output channels, K = 27 taps x input channels) on
// v_mfma_f32_16x16x32_bf16: each wavefront owns 32 cells x up to 64 output
// channels, K advances 32 at a time (a lane's 8 K values are 8 consecutive
// channels of one tap: one 16-byte load), FP32 accumulation, bias and ReLU
// fused into the store.  The input gradient is the same kernel on the FP32
// output gradient with flipped, transposed weights; weight gradients are an
// FP32 reduction over cells in fixed-order chunks (deterministic).
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

constexpr int kConvWaves = 4;             // wavefronts per workgroup, 32 cells each
constexpr int kChunk = 8192;              // cells per weight-gradient partial
constexpr int kWgBlock = 64;              // cells staged in LDS per step of the weight gradient

struct ConvArgs {
    const void *in;       // [cell][cin_s], bf16 or FP32
    int in_f32, cin_s, lg_cin;
    int nx, ny, nz;
    long ncell;
    const u16 *w;         // packed [cop][kp] bf16
    int kp;
    const float *bias;    // [co] or null
    void *out;            // [cell][out_s], bf16 or FP32
    int out_f32, out_s, co, relu;
};

__device__ __forceinline__ bf16x8 load8(const ConvArgs &a, long cell, int c0) {
    if (!a.in_f32) {
        u32x4 v = gld((const u32x4 *)((const u16 *)a.in + cell * a.cin_s + c0), 0);
        return __builtin_bit_cast(bf16x8, v);
    }
    const f32x4 *p = (const f32x4 *)((const float *)a.in + cell * a.cin_s + c0);
    f32x4 lo = gld(p, 0), hi = gld(p, 1);
    u32x4 v;
    v[0] = (uint32_t)f2bf(lo[0]) | ((uint32_t)f2bf(lo[1]) << 16);
    v[1] = (uint32_t)f2bf(lo[2]) | ((uint32_t)f2bf(lo[3]) << 16);
    v[2] = (uint32_t)f2bf(hi[0]) | ((uint32_t)f2bf(hi[1]) << 16);
    v[3] = (uint32_t)f2bf(hi[2]) | ((uint32_t)f2bf(hi[3]) << 16);
    return __builtin_bit_cast(bf16x8, v);
}

template <int NB>
__global__ void __launch_bounds__(64 * kConvWaves) k_conv(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long vbase = ((long)blockIdx.x * kConvWaves + wave) * 32;
    const int r = lane & 15, kq = lane >> 4;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long nxy = (long)nx * ny;
    int vi[2], vj[2], vk[2];
    bool vok[2];
#pragma unroll
    for (int rb = 0; rb < 2; rb++) {
        const long v = vbase + rb * 16 + r;
        vok[rb] = v < a.ncell;
        const long vv = vok[rb] ? v : 0;
        vk[rb] = (int)(vv / nxy);
        const long rem = vv - (long)vk[rb] * nxy;
        vj[rb] = (int)(rem / nx);
        vi[rb] = (int)(rem - (long)vj[rb] * nx);
    }
    f32x4 acc[2][NB];
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int nb = 0; nb < NB; nb++) acc[rb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u});
    for (int k0 = kq * 8; k0 < a.kp; k0 += 32) {
        const int tap = k0 >> a.lg_cin;
        const int c0 = k0 & (a.cin_s - 1);
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
        bf16x8 A[2];
#pragma unroll
        for (int rb = 0; rb < 2; rb++) {
            const int ii = vi[rb] + dx - 1, jj = vj[rb] + dy - 1, kk = vk[rb] + dz - 1;
            const bool ok = tap < 27 && vok[rb] && ii >= 0 && ii < nx && jj >= 0 && jj < ny && kk >= 0 && kk < nz;
            A[rb] = ok ? load8(a, ii + nx * (jj + (long)ny * kk), c0) : zero;
        }
        bf16x8 B[NB];
#pragma unroll
        for (int nb = 0; nb < NB; nb++)
            B[nb] = __builtin_bit_cast(bf16x8, gld((const u32x4 *)(a.w + (long)(nb * 16 + r) * a.kp + k0), 0));
#pragma unroll
        for (int rb = 0; rb < 2; rb++)
#pragma unroll
            for (int nb = 0; nb < NB; nb++)
                acc[rb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[rb], B[nb], acc[rb][nb], 0, 0, 0);
    }
    // lane holds rows 4*kq .. 4*kq+3 (cells) of column r (output channel)
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int nb = 0; nb < NB; nb++) {
            const int col = nb * 16 + r;
            if (col >= a.out_s) continue;
            const float bv = (a.bias && col < a.co) ? gld(a.bias, col) : 0.0f;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const long v = vbase + rb * 16 + kq * 4 + e;
                if (v >= a.ncell) continue;
                float val = 0.0f;
                if (col < a.co) {
                    val = acc[rb][nb][e] + bv;
                    if (a.relu) val = fmaxf(val, 0.0f);
                }
                if (a.out_f32) gst((float *)a.out, v * a.out_s + col, val);
                else gst((u16 *)a.out, v * a.out_s + col, f2bf(val));
            }
        }
}

// packed bf16 weights of one convolution: forward [cop][kp] with
// k = tap * cin_s + ci; transposed (for the input gradient) [cip16][kpT]
// with k = tap' * cout_s + co and tap' = 26 - tap
__global__ void k_pack(const float *__restrict__ w, int ci, int co, int cin_s, int kp, int cop, u16 *__restrict__ wf,
                       int cout_s, int kpT, int cipT, u16 *__restrict__ wt) {
    const long n1 = (long)cop * kp, n2 = (long)cipT * kpT;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n1 + n2; q += (long)gridDim.x * blockDim.x) {
        if (q < n1) {
            const int n = (int)(q / kp), k = (int)(q % kp);
            const int tap = k / cin_s, c = k % cin_s;
            float v = 0.0f;
            if (n < co && c < ci && tap < 27) v = gld(w, ((long)n * 27 + tap) * ci + c);
            gst(wf, q, f2bf(v));
        } else {
            const long q2 = q - n1;
            const int n = (int)(q2 / kpT), k = (int)(q2 % kpT);
            const int tp = k / cout_s, c = k % cout_s;
            float v = 0.0f;
            if (n < ci && c < co && tp < 27) v = gld(w, ((long)c * 27 + (26 - tp)) * ci + n);
            gst(wt, q2, f2bf(v));
        }
    }
}

// Weight and bias gradient partials: workgroup (chunk, tap) sums
// x[cell + offset(tap)][ci] * dy[cell][co] over its chunk of cells in a fixed
// order; the bias partial (sum of dy) comes from the tap-0 workgroups.
struct WgArgs {
    const u16 *x;
    int xs, ci;
    const float *dy;
    int dys, co;
    int nx, ny, nz;
    long ncell;
    float *part, *partb;
};

__global__ void __launch_bounds__(256) k_wgrad(WgArgs a) {
    extern __shared__ float wlds[];
    const int tap = blockIdx.y;
    const long c_begin = (long)blockIdx.x * kChunk;
    const long c_end = min(c_begin + (long)kChunk, a.ncell);
    const int ci = a.ci, co = a.co, nout = ci * co;
    float *xsb = wlds;                       // [kWgBlock][ci]
    float *dyb = wlds + kWgBlock * ci;       // [kWgBlock][co]
    float *red = dyb + kWgBlock * co;        // [256]
    const int groups = nout >= 256 ? 1 : 256 / nout;
    const int nq = (nout + 255) / 256;
    const int t = threadIdx.x;
    const int g = nout >= 256 ? 0 : t / nout;
    const int dz = tap / 9 - 1, dyo = (tap / 3) % 3 - 1, dxo = tap % 3 - 1;
    const long nxy = (long)a.nx * a.ny;
    float acc[16] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float bacc = 0.0f;
    for (long b0 = c_begin; b0 < c_end; b0 += kWgBlock) {
        for (int q = t; q < kWgBlock * ci; q += 256) {
            const int vv = q / ci, c = q % ci;
            const long v = b0 + vv;
            float val = 0.0f;
            if (v < c_end) {
                const int k = (int)(v / nxy);
                const long rem = v - (long)k * nxy;
                const int j = (int)(rem / a.nx), i = (int)(rem - (long)j * a.nx);
                const int ii = i + dxo, jj = j + dyo, kk = k + dz;
                if (ii >= 0 && ii < a.nx && jj >= 0 && jj < a.ny && kk >= 0 && kk < a.nz)
                    val = bf2f(gld(a.x, (ii + a.nx * (jj + (long)a.ny * kk)) * a.xs + c));
            }
            lst(xsb, q, val);
        }
        for (int q = t; q < kWgBlock * co; q += 256) {
            const int vv = q / co, c = q % co;
            const long v = b0 + vv;
            lst(dyb, q, v < c_end ? gld(a.dy, v * a.dys + c) : 0.0f);
        }
        __syncthreads();
        if (nout >= 256) {
            for (int qq = 0; qq < nq; qq++) {
                const int o = t + 256 * qq;
                if (o >= nout) break;
                const int oc = o / ci, ic = o % ci;
                float s = acc[qq];
                for (int vv = 0; vv < kWgBlock; vv++) s += lld(xsb, vv * ci + ic) * lld(dyb, vv * co + oc);
                acc[qq] = s;
            }
        } else if (t < groups * nout) {
            const int o = t % nout, oc = o / ci, ic = o % ci;
            float s = acc[0];
            for (int vv = g; vv < kWgBlock; vv += groups) s += lld(xsb, vv * ci + ic) * lld(dyb, vv * co + oc);
            acc[0] = s;
        }
        if (tap == 0 && t < co) {
            float s = bacc;
            for (int vv = 0; vv < kWgBlock; vv++) s += lld(dyb, vv * co + t);
            bacc = s;
        }
        __syncthreads();
    }
    float *out = a.part + ((long)blockIdx.x * 27 + tap) * nout;
    if (nout >= 256) {
        for (int qq = 0; qq < nq; qq++) {
            const int o = t + 256 * qq;
            if (o < nout) gst(out, o, acc[qq]);
        }
    } else {
        // fixed-order sum over the groups
        lst(red, t, t < groups * nout ? acc[0] : 0.0f);
        __syncthreads();
        if (t < nout) {
            float s = 0.0f;
            for (int q = 0; q < groups; q++) s += lld(red, q * nout + t);
            gst(out, t, s);
        }
    }
    if (tap == 0 && t < co) gst(a.partb, (long)blockIdx.x * co + t, bacc);
}

// dW[co][tap][ci] (the flat parameter layout) and db[co] from the partials,
// summed over chunks in order
__global__ void k_wgrad_reduce(const float *__restrict__ part, const float *__restrict__ partb, int nchunk, int ci, int co,
                               float *__restrict__ dw, float *__restrict__ db) {
    const int nout = ci * co;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < 27 * nout) {
        const int tap = q / nout, o = q % nout, oc = o / ci, ic = o % ci;
        float s = 0.0f;
        for (int c = 0; c < nchunk; c++) s += gld(part, ((long)c * 27 + tap) * nout + o);
        gst(dw, ((long)oc * 27 + tap) * ci + ic, s);
    } else if (q < 27 * nout + co) {
        const int oc = q - 27 * nout;
        float s = 0.0f;
        for (int c = 0; c < nchunk; c++) s += gld(partb, (long)c * co + oc);
        gst(db, oc, s);
    }
}

// ---------------------------------------------------------- elementwise
// mean of the 2x2x2 children, rounded to bf16
__global__ void k_pool(const u16 *__restrict__ in, u16 *__restrict__ out, int nx, int ny, int nz, int cs) {
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
                    s += bf2f(gld(in, ((2 * I + ii) + nx * ((2 * J + jj) + (long)ny * (2 * K + kk))) * cs + c));
        gst(out, q, f2bf(s * 0.125f));
    }
}

// s = upsample(t) + e (nearest), rounded to bf16
__global__ void k_upadd(const u16 *__restrict__ t, const u16 *__restrict__ e, u16 *__restrict__ s, int nx, int ny, int nz,
                        int cs) {
    const long n = (long)nx * ny * nz * cs;
    const int cx = nx / 2, cy = ny / 2;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int c = (int)(q % cs);
        const long v = q / cs;
        const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((long)nx * ny));
        const long pv = (i / 2) + cx * ((j / 2) + (long)cy * (k / 2));
        gst(s, q, f2bf(bf2f(gld(t, pv * cs + c)) + bf2f(gld(e, q))));
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

// [cell][cin] bf16 -> [cell][cs] bf16 with zero channels
__global__ void k_in_pad(const u16 *__restrict__ in, int cin, u16 *__restrict__ out, int cs, long ncell) {
    const long n = ncell * cs;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int c = (int)(q % cs);
        gst(out, q, c < cin ? gld(in, (q / cs) * cin + c) : (u16)0);
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

struct Conv {
    int ci, co, cis, cos, kp, cop, kpT, cipT;
    long woff, boff;
    DevBuf<u16> wf, wt;
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
    DevBuf<float> part, partb;
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
    long pmax = 0, pbmax = 0;
    for (auto &c : N.convs) {
        // the weight gradient of a convolution runs at the resolution of its input
        pmax = std::max(pmax, (long)c.ci * c.co * 27);
        pbmax = std::max(pbmax, (long)c.co);
    }
    const long nch = (n0 + kChunk - 1) / kChunk;
    N.part.alloc((size_t)nch * pmax);
    N.partb.alloc((size_t)nch * pbmax);
    N.mse_part.alloc(grid_for(n0));
    N.gx = nx; N.gy = ny; N.gz = nz;
}

static void pack_all(vd_ctx *ctx, Net &N) {
    for (auto &c : N.convs)
        k_pack<<<grid_for((long)c.cop * c.kp + (long)c.cipT * c.kpT), 256, 0, ctx->stream>>>(
            N.params.p + c.woff, c.ci, c.co, c.cis, c.kp, c.cop, c.wf.p, c.cos, c.kpT, c.cipT, c.wt.p);
    VD_HIP(hipGetLastError());
    N.packed = true;
}

// one convolution; transposed = input-gradient form (in: FP32 gradient with
// cos channels, out: FP32 with cis channels)
static void run_conv(vd_ctx *ctx, Net &N, const Conv &c, const Level &V, const void *in, bool in_f32, void *out, bool out_f32,
                     int out_s, bool relu, bool transposed) {
    ConvArgs a;
    a.in = in; a.in_f32 = in_f32 ? 1 : 0;
    a.cin_s = transposed ? c.cos : c.cis;
    a.lg_cin = lg2(a.cin_s);
    a.nx = V.nx; a.ny = V.ny; a.nz = V.nz; a.ncell = V.n;
    a.w = transposed ? c.wt.p : c.wf.p;
    a.kp = transposed ? c.kpT : c.kp;
    a.bias = transposed ? nullptr : N.params.p + c.boff;
    a.out = out; a.out_f32 = out_f32 ? 1 : 0; a.out_s = out_s;
    a.co = transposed ? c.ci : c.co;
    a.relu = relu ? 1 : 0;
    const int cop = transposed ? c.cipT : c.cop;
    const int nb = cop / 16;
    const long nblk = (V.n + 32 * kConvWaves - 1) / (32 * kConvWaves);
    VD_CHECK(nb >= 1 && nb <= 4, "internal: conv width");
    VD_CHECK(out_s <= cop, "internal: conv output stride");
    timed(ctx, "nn_conv", 0.0, [&] {
        switch (nb) {
        case 1: k_conv<1><<<nblk, 64 * kConvWaves, 0, ctx->stream>>>(a); break;
        case 2: k_conv<2><<<nblk, 64 * kConvWaves, 0, ctx->stream>>>(a); break;
        case 3: k_conv<3><<<nblk, 64 * kConvWaves, 0, ctx->stream>>>(a); break;
        default: k_conv<4><<<nblk, 64 * kConvWaves, 0, ctx->stream>>>(a); break;
        }
    });
}

static void run_wgrad(vd_ctx *ctx, Net &N, const Conv &c, const Level &V, const u16 *x, const float *dy) {
    WgArgs a;
    a.x = x; a.xs = c.cis; a.ci = c.ci;
    a.dy = dy; a.dys = c.cos; a.co = c.co;
    a.nx = V.nx; a.ny = V.ny; a.nz = V.nz; a.ncell = V.n;
    a.part = N.part.p; a.partb = N.partb.p;
    const int nch = (int)((V.n + kChunk - 1) / kChunk);
    const size_t lds = sizeof(float) * ((size_t)kWgBlock * (c.ci + c.co) + 256);
    timed(ctx, "nn_wgrad", 0.0, [&] {
        k_wgrad<<<dim3(nch, 27), 256, lds, ctx->stream>>>(a);
        const int tot = 27 * c.ci * c.co + c.co;
        k_wgrad_reduce<<<(tot + 255) / 256, 256, 0, ctx->stream>>>(N.part.p, N.partb.p, nch, c.ci, c.co, N.grads.p + c.woff,
                                                                  N.grads.p + c.boff);
    });
}

static void forward(vd_ctx *ctx, Net &N, const u16 *in_cin) {
    if (!N.packed) pack_all(ctx, N);
    const int L = N.cfg.levels;
    hipStream_t s = ctx->stream;
    Level &V0 = N.lv[0];
    const int cin_s = pow2pad(N.cfg.cin);
    k_in_pad<<<grid_for(V0.n * cin_s), 256, 0, s>>>(in_cin, N.cfg.cin, V0.in.p, cin_s, V0.n);
    for (int l = 0; l < L; l++) {
        Level &V = N.lv[l];
        const Conv &ca = N.convs[N.enc_a[l]], &cb = N.convs[N.enc_b[l]];
        if (l > 0) {
            const Level &P = N.lv[l - 1];
            k_pool<<<grid_for(V.n * ca.cis), 256, 0, s>>>(P.e.p, V.in.p, P.nx, P.ny, P.nz, ca.cis);
        }
        run_conv(ctx, N, ca, V, V.in.p, false, V.a.p, false, ca.cos, true, false);
        run_conv(ctx, N, cb, V, V.a.p, false, V.e.p, false, cb.cos, true, false);
    }
    const u16 *d = N.lv[L - 1].e.p;
    for (int l = L - 2; l >= 0; l--) {
        Level &V = N.lv[l], &C = N.lv[l + 1];
        const Conv &cu = N.convs[N.up[l]], &cd = N.convs[N.dec[l]];
        run_conv(ctx, N, cu, C, d, false, C.t.p, false, cu.cos, true, false);
        k_upadd<<<grid_for(V.n * cu.cos), 256, 0, s>>>(C.t.p, V.e.p, V.s.p, V.nx, V.ny, V.nz, cu.cos);
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
        c.ci = sh.first; c.co = sh.second;
        c.cis = pow2pad(c.ci); c.cos = pow2pad(c.co);
        c.kp = (27 * c.cis + 31) / 32 * 32;
        c.cop = std::max((c.co + 15) / 16 * 16, c.cos);
        c.kpT = (27 * c.cos + 31) / 32 * 32;
        c.cipT = std::max((c.ci + 15) / 16 * 16, c.cis);
        c.woff = off;
        off += (long)c.co * 27 * c.ci;
        c.boff = off;
        off += c.co;
        c.wf.alloc((size_t)c.cop * c.kp);
        c.wt.alloc((size_t)c.cipT * c.kpT);
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
    c.ci = ci; c.co = co;
    c.cis = pow2pad(ci); c.cos = pow2pad(co);
    c.kp = (27 * c.cis + 31) / 32 * 32;
    c.cop = std::max((co + 15) / 16 * 16, c.cos);
    c.kpT = (27 * c.cos + 31) / 32 * 32;
    c.cipT = std::max((ci + 15) / 16 * 16, c.cis);
    c.woff = 0;
    c.boff = (long)co * 27 * ci;
    c.wf.alloc((size_t)c.cop * c.kp);
    c.wt.alloc((size_t)c.cipT * c.kpT);
    N.params.alloc(N.nparam);
    N.grads.alloc(N.nparam);
    hipStream_t s = ctx->stream;
    VD_HIP(hipMemcpyAsync(N.params.p, w, sizeof(float) * c.boff, hipMemcpyDeviceToDevice, s));
    if (b) VD_HIP(hipMemcpyAsync(N.params.p + c.boff, b, sizeof(float) * co, hipMemcpyDeviceToDevice, s));
    else VD_HIP(hipMemsetAsync(N.params.p + c.boff, 0, sizeof(float) * co, s));
    k_pack<<<grid_for((long)c.cop * c.kp + (long)c.cipT * c.kpT), 256, 0, s>>>(N.params.p, ci, co, c.cis, c.kp, c.cop, c.wf.p,
                                                                               c.cos, c.kpT, c.cipT, c.wt.p);
    Level V;
    V.nx = g->nx; V.ny = g->ny; V.nz = g->nz; V.n = n;
    DevBuf<u16> xin;
    xin.alloc((size_t)n * c.cis);
    k_in_pad<<<grid_for(n * c.cis), 256, 0, s>>>(x, ci, xin.p, c.cis, n);
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
        const long nch = (n + kChunk - 1) / kChunk;
        N.part.alloc((size_t)nch * 27 * ci * co);
        N.partb.alloc((size_t)nch * co);
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
