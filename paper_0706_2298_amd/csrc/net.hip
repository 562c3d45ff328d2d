// Kernels of the start-field network and its training: periodic 3^4
// convolutions (forward, backward to the input, backward to the weights),
// the maps between output channels and quark fields, the block deficit loss
// of eq. (3.15) with its gradient, and the Adam update.
//
// Activations are FP32 planes [C][V] in canonical site order (x0 slowest),
// so a tap's neighbour is a fixed shift of the site index up to the periodic
// wrap. Weights are [81][Cin][Cout], tap t = sum_mu (o_mu + 1) 3^(3 - mu) for
// the offset o in {-1,0,1}^4. Quark fields are native FP64 fields (common.h).
#include <mutex>

#include "internal.h"

namespace dfl {

namespace {

constexpr int kCO = 16;        // output channels per workgroup of the convolution
constexpr int kWT = 64;        // output channels per workgroup of the weight gradient
constexpr int kWS = 64;        // sites per LDS tile of the weight gradient
constexpr int kMaxCin = 96;

struct Lat {
    int L[4];
    long str[4];  // canonical strides (x3 fastest)
    long V;
};

// delta[mu][o+1]: index shift of the neighbour x + o mu_hat of site i
__device__ inline void tap_shifts(const Lat& lt, long i, int sign, long delta[4][3])
{
    long rest = i;
    int x[4];
    for (int mu = 3; mu >= 0; --mu) {
        x[mu] = (int)(rest % lt.L[mu]);
        rest /= lt.L[mu];
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
        for (int o = -1; o <= 1; ++o) {
            int y = x[mu] + sign * o;
            if (y < 0)
                y += lt.L[mu];
            if (y >= lt.L[mu])
                y -= lt.L[mu];
            delta[mu][o + 1] = (long)(y - x[mu]) * lt.str[mu];
        }
    }
}

// canonical index of site x3 on the x3 line `line` = (x0 L1 + x1) L2 + x2
__device__ inline long base_site(const Lat& lt, long line, int x3) { return line * lt.L[3] + x3; }

__device__ inline float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float silu_grad_f(float z)
{
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// out[oc][i] = bias[oc] + sum_t sum_ic Wt(t, ic, oc) in[ic][i + s*o_t]
//   forward (TRANS = false, s = +1): Wt(t, ic, oc) = W[t][ic][oc], nic = Cin
//   input gradient (TRANS = true, s = -1): Wt(t, ic, oc) = W[t][oc][ic], nic = Cout of W
// Epilogue: forward stores z and optionally a = silu(z); the input gradient
// is optionally multiplied by silu'(zprev[oc][i]).
template <bool TRANS>
__global__ __launch_bounds__(256) void k_conv(Lat lt, const float* __restrict__ in, int nic,
                                              const float* __restrict__ W, int w_cin, int w_cout,
                                              const float* __restrict__ bias, int noc, float* __restrict__ out,
                                              float* __restrict__ act, const float* __restrict__ zprev)
{
    __shared__ float4 ws[kMaxCin * kCO / 4 > 576 * kCO / 4 ? kMaxCin * kCO / 4 : 576 * kCO / 4];
    const long V = lt.V;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int oc0 = blockIdx.y * kCO;
    long dl[4][3];
    if (i < V)
        tap_shifts(lt, i, TRANS ? -1 : 1, dl);
    float acc[kCO];
#pragma unroll
    for (int j = 0; j < kCO; ++j)
        acc[j] = (bias && oc0 + j < noc) ? bias[oc0 + j] : 0.f;
    float* wsf = reinterpret_cast<float*>(ws);
    for (int t = 0; t < 81; ++t) {
        __syncthreads();
        for (int e = threadIdx.x; e < nic * kCO; e += blockDim.x) {
            int ic, j;
            if (TRANS) {
                ic = e % nic;
                j = e / nic;
            } else {
                ic = e / kCO;
                j = e % kCO;
            }
            float w = 0.f;
            if (oc0 + j < noc)
                w = TRANS ? W[((long)t * w_cin + oc0 + j) * w_cout + ic] : W[((long)t * w_cin + ic) * w_cout + oc0 + j];
            wsf[ic * kCO + j] = w;
        }
        __syncthreads();
        if (i < V) {
            const int o0 = t / 27, o1 = (t / 9) % 3, o2 = (t / 3) % 3, o3 = t % 3;
            const long nb = i + dl[0][o0] + dl[1][o1] + dl[2][o2] + dl[3][o3];
            const float* src = in + nb;
            for (int ic = 0; ic < nic; ++ic) {
                const float x = src[(long)ic * V];
#pragma unroll
                for (int q = 0; q < kCO / 4; ++q) {
                    const float4 w = ws[ic * (kCO / 4) + q];
                    acc[4 * q] += x * w.x;
                    acc[4 * q + 1] += x * w.y;
                    acc[4 * q + 2] += x * w.z;
                    acc[4 * q + 3] += x * w.w;
                }
            }
        }
    }
    if (i >= V)
        return;
#pragma unroll
    for (int j = 0; j < kCO; ++j) {
        if (oc0 + j >= noc)
            continue;
        float v = acc[j];
        if (TRANS && zprev)
            v *= silu_grad_f(zprev[(long)(oc0 + j) * V + i]);
        out[(long)(oc0 + j) * V + i] = v;
        if (!TRANS && act)
            act[(long)(oc0 + j) * V + i] = silu_f(v);
    }
}

// The same map on the matrix cores (v_mfma_f32_16x16x4f32, FP32 products
// and sums), as a GEMM per tap: out[oc][x] += sum_ic Wt(t, ic, oc) in[ic][x + s o_t].
// Workgroup: 32 consecutive sites along x3 (L3 % 32 == 0) and 32 output
// channels; wavefront w computes the 16 x 16 tile (channels (w / 2) * 16..,
// sites (w % 2) * 16..). For each of the 27 neighbour lines (o0, o1, o2) and
// each chunk of kMC input channels, the line segment with its +-1 halo along
// x3 and the weights of the three taps o3 = -1, 0, 1 are staged in LDS; the
// three taps then read the segment at shifts of one site. Operand layout of
// the 16x16x4 instruction: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds C[4 (l / 16) + i][l % 16], i < 4.
// Measured on MI355X: 44-50 TFLOP/s per layer on 64 x 32^3, 15% faster than
// k_conv; 16-site segments (for L3 = 16) ran three times slower than k_conv
// and two channel tiles per wavefront did not help, so only this shape is
// used and other lattices take k_conv.
constexpr int kMC = 32;  // input channels per LDS chunk
constexpr int kXS = 48;  // LDS row stride of the staged segment (34 used; 48 = 16 mod 32 banks)
template <bool TRANS>
__global__ __launch_bounds__(256) void k_conv_mfma(Lat lt, const float* __restrict__ in, int nic,
                                                   const float* __restrict__ W, int w_cin, int w_cout,
                                                   const float* __restrict__ bias, int noc, float* __restrict__ out,
                                                   float* __restrict__ act, const float* __restrict__ zprev)
{
    constexpr int TS = 32;              // sites per workgroup
    constexpr int OCT = 32;             // output channels per workgroup
    constexpr int WS = OCT + 16;        // LDS row stride of the weights (16 mod 32 banks)
    constexpr int NST = TS / 16;        // site tiles per workgroup
    __shared__ float xs[kMC][kXS];
    __shared__ float ws[3][kMC][WS];
    const int sgn = TRANS ? -1 : 1;
    const long V = lt.V;
    const int L3 = lt.L[3];
    const long seg = blockIdx.x;                          // segment of TS sites of one x3 line
    const long line = seg / (L3 / TS);
    const int x3_0 = (int)(seg - line * (L3 / TS)) * TS;
    int x[3];
    {
        long r = line;
        x[2] = (int)(r % lt.L[2]);
        r /= lt.L[2];
        x[1] = (int)(r % lt.L[1]);
        x[0] = (int)(r / lt.L[1]);
    }
    const int oc0 = blockIdx.y * OCT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ot = w / NST, st = w % NST;
    const int kr = lane >> 4, kc = lane & 15;             // k row and column of this lane's operands
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int l = 0; l < 27; ++l) {
        const int o[3] = {l / 9 - 1, (l / 3) % 3 - 1, l % 3 - 1};
        long base = 0;  // canonical index of (y0, y1, y2, 0)
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            int y = x[mu] + sgn * o[mu];
            y = y < 0 ? y + lt.L[mu] : (y >= lt.L[mu] ? y - lt.L[mu] : y);
            base += (long)y * lt.str[mu];
        }
        for (int c0 = 0; c0 < nic; c0 += kMC) {
            __syncthreads();  // the previous chunk's operands are consumed
            for (int e = threadIdx.x; e < kMC * (TS + 2); e += 256) {
                const int ic = e / (TS + 2), j = e - ic * (TS + 2);
                int y3 = x3_0 - 1 + j;
                y3 = y3 < 0 ? y3 + L3 : (y3 >= L3 ? y3 - L3 : y3);
                xs[ic][j] = c0 + ic < nic ? in[(long)(c0 + ic) * V + base + y3] : 0.f;
            }
            for (int e = threadIdx.x; e < 3 * kMC * OCT; e += 256) {
                const int q = e / (kMC * OCT), r = e - q * (kMC * OCT);
                const int ic = r / OCT, c = r - ic * OCT;
                const int t = l * 3 + q;  // tap of (o0, o1, o2, o3 = q - 1)
                const int ci = c0 + ic, co = oc0 + c;
                float v = 0.f;
                if (ci < nic && co < noc)
                    v = TRANS ? W[((long)t * w_cin + co) * w_cout + ci] : W[((long)t * w_cin + ci) * w_cout + co];
                ws[q][ic][c] = v;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int sh = 1 + sgn * (q - 1);  // segment column of site 0 for o3 = q - 1
#pragma unroll
                for (int k0 = 0; k0 < kMC; k0 += 4) {
                    const float a = ws[q][k0 + kr][ot * 16 + kc];
                    const float b = xs[k0 + kr][st * 16 + kc + sh];
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
                }
            }
        }
    }
    const long site = base_site(lt, line, x3_0 + st * 16 + kc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int oc = oc0 + ot * 16 + 4 * kr + i;
        if (oc >= noc)
            continue;
        float v = acc[i] + (bias ? bias[oc] : 0.f);
        if (TRANS && zprev)
            v *= silu_grad_f(zprev[(long)oc * V + site]);
        out[(long)oc * V + site] = v;
        if (!TRANS && act)
            act[(long)oc * V + site] = silu_f(v);
    }
}

// Forward map with BF16 operands on the matrix cores: inputs and weights
// rounded to BF16 (nearest even), products summed in FP32
// (v_mfma_f32_16x16x32_bf16), bias and activation in FP32. The weights come
// pre-converted as Wb[t][oc][ic] (ic padded to a multiple of 32 and oc to
// the channel tile with zeros), so a tap's 32-channel chunk is a straight
// 16-byte copy into LDS. Workgroup: kBNL consecutive x2 lines of kBTS sites
// along x3 (one line per wavefront) and 16 OT output channels; every
// wavefront keeps OT x 2 tiles of 16 x 16 accumulators, so one staged
// operand row feeds two (weights) or OT (inputs) instructions. For each of
// the 27 neighbour line offsets (o0, o1, o2) and each 32-channel chunk the
// four lines' segments with their +-1 halo along x3 and the three taps'
// weights (o3 = -1, 0, 1) are staged; the taps read the segments at shifts
// of one site. Lane l supplies A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j < 8 (the contraction index is summed, so
// only its being the same for A and B matters) and holds
// C[4 (l / 16) + i][l % 16], i < 4.
// round-to-nearest-even float -> bfloat16 bits (finite inputs)
__device__ inline uint32_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

constexpr int kBTS = 32;       // sites per line segment
constexpr int kBNL = 4;        // x2 lines per workgroup (one per wavefront)
constexpr int kBK = 32;        // input channels per chunk (the instruction's K)
constexpr int kBRow = kBK + 8; // LDS row stride in BF16 elements (80 bytes)
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

template <int OT>
__global__ __launch_bounds__(256) void k_conv_bf16(Lat lt, const float* __restrict__ in, int cin, int cinP,
                                                   const uint16_t* __restrict__ Wb, int coutP,
                                                   const float* __restrict__ bias, int cout, float* __restrict__ out,
                                                   float* __restrict__ act)
{
    constexpr int OCT = 16 * OT;
    __shared__ __attribute__((aligned(16))) uint16_t xs[kBNL][kBTS + 2][kBRow];
    __shared__ __attribute__((aligned(16))) uint16_t ws[3][OCT][kBRow];
    typedef float f4 __attribute__((ext_vector_type(4)));
    const long V = lt.V;
    const int n_oct = coutP / OCT;
    const long grp = blockIdx.x / n_oct;  // channel tiles of one site group are adjacent
    const int oc0 = (int)(blockIdx.x - grp * n_oct) * OCT;
    const int nseg = lt.L[3] / kBTS, ngx2 = lt.L[2] / kBNL;
    long r = grp;
    const int seg = (int)(r % nseg);
    r /= nseg;
    const int x2g = (int)(r % ngx2) * kBNL;
    r /= ngx2;
    const int x1 = (int)(r % lt.L[1]);
    const int x0 = (int)(r / lt.L[1]);
    const int x3_0 = seg * kBTS;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kr = lane >> 4, kc = lane & 15;
    f4 acc[OT][2];
#pragma unroll
    for (int ot = 0; ot < OT; ++ot)
        acc[ot][0] = acc[ot][1] = f4{0.f, 0.f, 0.f, 0.f};
    for (int l = 0; l < 27; ++l) {
        const int o0 = l / 9 - 1, o1 = (l / 3) % 3 - 1, o2 = l % 3 - 1;
        int y0 = x0 + o0, y1 = x1 + o1;
        y0 = y0 < 0 ? y0 + lt.L[0] : (y0 >= lt.L[0] ? y0 - lt.L[0] : y0);
        y1 = y1 < 0 ? y1 + lt.L[1] : (y1 >= lt.L[1] ? y1 - lt.L[1] : y1);
        const long base01 = (long)y0 * lt.str[0] + (long)y1 * lt.str[1];
        for (int c0 = 0; c0 < cinP; c0 += kBK) {
            __syncthreads();  // the previous chunk's operands are consumed
            for (int e = threadIdx.x; e < kBNL * kBK * (kBTS + 2); e += 256) {
                const int j = e % (kBTS + 2);
                const int rest = e / (kBTS + 2);
                const int ic = rest % kBK, ln = rest / kBK;
                int y2 = x2g + ln + o2;
                y2 = y2 < 0 ? y2 + lt.L[2] : (y2 >= lt.L[2] ? y2 - lt.L[2] : y2);
                int y3 = x3_0 - 1 + j;
                y3 = y3 < 0 ? y3 + lt.L[3] : (y3 >= lt.L[3] ? y3 - lt.L[3] : y3);
                const float v = c0 + ic < cin ? in[(long)(c0 + ic) * V + base01 + (long)y2 * lt.str[2] + y3] : 0.f;
                xs[ln][j][ic] = (uint16_t)bf16_bits(v);
            }
            for (int e = threadIdx.x; e < 3 * OCT * (kBK / 8); e += 256) {
                const int v8 = e % (kBK / 8);
                const int rest = e / (kBK / 8);
                const int oc = rest % OCT, q = rest / OCT;
                const long t = l * 3 + q;  // tap of (o0, o1, o2, o3 = q - 1)
                *reinterpret_cast<u16x8*>(&ws[q][oc][8 * v8]) =
                    *reinterpret_cast<const u16x8*>(Wb + (t * coutP + oc0 + oc) * cinP + c0 + 8 * v8);
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                // the neighbour x3 + (q - 1) of segment site i sits in staged column i + q
                bf16x8 b[2];
#pragma unroll
                for (int st = 0; st < 2; ++st)
                    b[st] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&xs[w][st * 16 + kc + q][8 * kr]));
#pragma unroll
                for (int ot = 0; ot < OT; ++ot) {
                    const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&ws[q][ot * 16 + kc][8 * kr]));
#pragma unroll
                    for (int st = 0; st < 2; ++st)
                        acc[ot][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[st], acc[ot][st], 0, 0, 0);
                }
            }
        }
    }
    const long line = ((long)x0 * lt.L[1] + x1) * lt.L[2] + x2g + w;
#pragma unroll
    for (int ot = 0; ot < OT; ++ot)
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const long site = base_site(lt, line, x3_0 + st * 16 + kc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int oc = oc0 + ot * 16 + 4 * kr + i;
                if (oc >= cout)
                    continue;
                const float v = acc[ot][st][i] + (bias ? bias[oc] : 0.f);
                out[(long)oc * V + site] = v;
                if (act)
                    act[(long)oc * V + site] = silu_f(v);
            }
        }
}

// Wb[t][oc][ic] = bf16(W[t][ic][oc]) on the padded [81][coutP][cinP] grid (zeros outside)
__global__ __launch_bounds__(256) void k_weights_bf16(const float* __restrict__ W, int cin, int cout, int cinP,
                                                      int coutP, uint16_t* __restrict__ Wb)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 81L * coutP * cinP)
        return;
    const int ic = (int)(e % cinP);
    const long rest = e / cinP;
    const int oc = (int)(rest % coutP);
    const long t = rest / coutP;
    const float v = (ic < cin && oc < cout) ? W[(t * cin + ic) * cout + oc] : 0.f;
    Wb[e] = (uint16_t)bf16_bits(v);
}

// Weight gradient, partial over a chunk of sites:
// part[chunk][t][ci][co] = sum_{y in chunk} in[ci][y + o_t] g[co][y].
// Workgroup (t, co tile of kWT, site chunk); thread (ci group, co), the
// tiles of g and of the shifted input staged in LDS kWS sites at a time.
__global__ __launch_bounds__(256) void k_conv_wgrad(Lat lt, const float* __restrict__ in, int cin,
                                                    const float* __restrict__ g, int cout, long chunk,
                                                    float* __restrict__ part)
{
    __shared__ float gs[kWS][kWT + 1];
    __shared__ float xs[kWS][kMaxCin + 1];
    const long V = lt.V;
    const int t = blockIdx.x;
    const int co0 = blockIdx.y * kWT;
    const long y0 = (long)blockIdx.z * chunk;
    const long y1 = y0 + chunk < V ? y0 + chunk : V;
    const int col = threadIdx.x % kWT, cg = threadIdx.x / kWT;  // 4 groups of ci
    const int cpt = (cin + 3) / 4;
    const int o0 = t / 27, o1 = (t / 9) % 3, o2 = (t / 3) % 3, o3 = t % 3;
    float acc[kMaxCin / 4];
#pragma unroll
    for (int c = 0; c < kMaxCin / 4; ++c)
        acc[c] = 0.f;
    for (long ys = y0; ys < y1; ys += kWS) {
        __syncthreads();
        for (int e = threadIdx.x; e < kWS * kWT; e += blockDim.x) {
            const int yy = e % kWS, cc = e / kWS;
            const long y = ys + yy;
            gs[yy][cc] = (y < y1 && co0 + cc < cout) ? g[(long)(co0 + cc) * V + y] : 0.f;
        }
        for (int e = threadIdx.x; e < kWS * cin; e += blockDim.x) {
            const int yy = e % kWS, ci = e / kWS;
            const long y = ys + yy;
            float v = 0.f;
            if (y < y1) {
                long dl[4][3];
                tap_shifts(lt, y, 1, dl);
                v = in[(long)ci * V + y + dl[0][o0] + dl[1][o1] + dl[2][o2] + dl[3][o3]];
            }
            xs[yy][ci] = v;
        }
        __syncthreads();
        for (int yy = 0; yy < kWS; ++yy) {
            const float gv = gs[yy][col];
#pragma unroll
            for (int c = 0; c < kMaxCin / 4; ++c)
                if (c < cpt && cg * cpt + c < cin)
                    acc[c] += xs[yy][cg * cpt + c] * gv;
        }
    }
    if (co0 + col >= cout)
        return;
    float* dst = part + ((long)blockIdx.z * 81 + t) * cin * cout;
#pragma unroll
    for (int c = 0; c < kMaxCin / 4; ++c) {
        const int ci = cg * cpt + c;
        if (c < cpt && ci < cin)
            dst[(long)ci * cout + co0 + col] = acc[c];
    }
}

// dW[e] = sum over chunks of part[chunk][e] (fixed order)
__global__ __launch_bounds__(256) void k_sum_chunks(const float* __restrict__ part, long n, int nchunk,
                                                    float* __restrict__ dW)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n)
        return;
    float s = 0.f;
    for (int q = 0; q < nchunk; ++q)
        s += part[(long)q * n + e];
    dW[e] = s;
}

// db[co] = sum_y g[co][y], one workgroup per channel
__global__ __launch_bounds__(256) void k_bias_grad(const float* __restrict__ g, long V, float* __restrict__ db)
{
    __shared__ float sh[16];
    const float* gc = g + (long)blockIdx.x * V;
    float s = 0.f;
    for (long y = threadIdx.x; y < V; y += blockDim.x)
        s += gc[y];
    s = block_sum(s, sh);
    if (threadIdx.x == 0)
        db[blockIdx.x] = s;
}

// canonical site index of native site s
__device__ inline long canon_of(const Geom& g, long s)
{
    int n[4], y[4], x[4];
    site_decompose(g, s, n, y);
    for (int mu = 0; mu < 4; ++mu)
        x[mu] = n[mu] * g.b[mu] + y[mu];
    return canon_index(g, x);
}

// x[c][i]: Re/Im of U_mu(x)[a][b] at channel ((mu*3 + a)*3 + b)*2 + r, then
// the 24 noise channels (noise [V][24], canonical)
__global__ __launch_bounds__(256) void k_features(Geom g, const c64* __restrict__ U64, const float* __restrict__ noise,
                                                  float* __restrict__ x)
{
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V)
        return;
    const long i = canon_of(g, s);
    for (int mu = 0; mu < 4; ++mu) {
        c64 u[9];
        for (int k = 0; k < 6; ++k)
            u[k] = U64[tidx(s, mu * 6 + k, 24)];
        for (int b = 0; b < 3; ++b)
            u[6 + b] = conjg(u[(b + 1) % 3] * u[3 + (b + 2) % 3] - u[(b + 2) % 3] * u[3 + (b + 1) % 3]);
        for (int k = 0; k < 9; ++k) {
            const int ch = 2 * (mu * 9 + k);
            x[(long)ch * g.V + i] = (float)u[k].re;
            x[(long)(ch + 1) * g.V + i] = (float)u[k].im;
        }
    }
    for (int k = 0; k < 24; ++k)
        x[(long)(72 + k) * g.V + i] = noise[i * 24 + k];
}

// field_l(x)[c] = out[(l*12 + c)*2][i] + i out[(l*12 + c)*2 + 1][i]
__global__ __launch_bounds__(256) void k_out_to_fields(Geom g, const float* __restrict__ out, int Ns,
                                                       c64* __restrict__ f)
{
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V)
        return;
    const long i = canon_of(g, s);
    const long F = 12 * g.V;
    for (int l = 0; l < Ns; ++l)
        for (int c = 0; c < 12; ++c) {
            const long ch = (long)(l * 12 + c) * 2;
            f[l * F + tidx(s, c, 12)] = c64{(double)out[ch * g.V + i], (double)out[(ch + 1) * g.V + i]};
        }
}

// dout[(l*12 + c)*2 + r][i] = 2 Re / 2 Im of grad_l(x)[c]  (real gradient of a
// real loss from its derivative with respect to conj(field))
__global__ __launch_bounds__(256) void k_fields_to_out(Geom g, const c64* __restrict__ gr, int Ns,
                                                       float* __restrict__ dout)
{
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V)
        return;
    const long i = canon_of(g, s);
    const long F = 12 * g.V;
    for (int l = 0; l < Ns; ++l)
        for (int c = 0; c < 12; ++c) {
            const long ch = (long)(l * 12 + c) * 2;
            const c64 v = gr[l * F + tidx(s, c, 12)];
            dout[ch * g.V + i] = (float)(2.0 * v.re);
            dout[(ch + 1) * g.V + i] = (float)(2.0 * v.im);
        }
}

// Per deflation block: G = Psi^+ Psi, C = Psi^+ T, Cholesky G = L L^+,
// Y = G^-1 C; writes Y[blk][l][k], tb2[blk][k] = ||t_k on the block||^2 and
// proj[blk][k] = Re(c_k^+ y_k). Entries are staged through LDS 64 at a time.
constexpr int kMaxLossN = 32;
constexpr int kLT = 64;  // staged entries

__global__ __launch_bounds__(256) void k_deficit_block(Geom g, const c64* __restrict__ Psi, int Ns,
                                                       const c64* __restrict__ T, int K, c64* __restrict__ Y,
                                                       double* __restrict__ tb2, double* __restrict__ proj,
                                                       int* __restrict__ flag)
{
    extern __shared__ double dyn[];
    c64* ps = reinterpret_cast<c64*>(dyn);              // [Ns][kLT + 1]
    c64* ts = ps + Ns * (kLT + 1);                      // [K][kLT + 1]
    c64* Gm = ts + K * (kLT + 1);                       // [Ns][Ns]
    c64* Cm = Gm + Ns * Ns;                             // [Ns][K]
    double* tn = reinterpret_cast<double*>(Cm + Ns * K);  // [K]
    const int blk = blockIdx.x;
    const long F = 12 * g.V;
    const int ne = 12 * g.Vb;
    // products: G (l <= m), C (l, k), ||t_k||^2
    const int nG = Ns * (Ns + 1) / 2, nC = Ns * K, np = nG + nC + K;
    c64 acc[8];
    int pid[8];
    int nmine = 0;
    for (int p = threadIdx.x; p < np && nmine < 8; p += blockDim.x)
        pid[nmine++] = p;
    for (int q = 0; q < 8; ++q)
        acc[q] = c64{0.0, 0.0};
    for (int e0 = 0; e0 < ne; e0 += kLT) {
        __syncthreads();
        for (int q = threadIdx.x; q < (Ns + K) * kLT; q += blockDim.x) {
            const int r = q / kLT, e = q % kLT;
            c64 v{0.0, 0.0};
            if (e0 + e < ne) {
                long idx;
                if ((g.Vb & (kTile - 1)) == 0)
                    idx = (long)blk * ne + e0 + e;
                else
                    idx = tidx((long)blk * g.Vb + (e0 + e) % g.Vb, (e0 + e) / g.Vb, 12);
                v = r < Ns ? Psi[(long)r * F + idx] : T[(long)(r - Ns) * F + idx];
            }
            if (r < Ns)
                ps[r * (kLT + 1) + e] = v;
            else
                ts[(r - Ns) * (kLT + 1) + e] = v;
        }
        __syncthreads();
        for (int q = 0; q < nmine; ++q) {
            const int p = pid[q];
            const c64 *u, *v;
            if (p < nG) {
                int l = 0, rem = p;
                while (rem >= Ns - l) {
                    rem -= Ns - l;
                    ++l;
                }
                u = ps + l * (kLT + 1);
                v = ps + (l + rem) * (kLT + 1);
            } else if (p < nG + nC) {
                const int l = (p - nG) / K, k = (p - nG) % K;
                u = ps + l * (kLT + 1);
                v = ts + k * (kLT + 1);
            } else {
                u = ts + (p - nG - nC) * (kLT + 1);
                v = u;
            }
            double re = acc[q].re, im = acc[q].im;
            for (int e = 0; e < kLT; ++e) {
                const c64 a = u[e], b = v[e];
                re += a.re * b.re + a.im * b.im;
                im += a.re * b.im - a.im * b.re;
            }
            acc[q] = c64{re, im};
        }
    }
    __syncthreads();
    for (int q = 0; q < nmine; ++q) {
        const int p = pid[q];
        if (p < nG) {
            int l = 0, rem = p;
            while (rem >= Ns - l) {
                rem -= Ns - l;
                ++l;
            }
            const int m = l + rem;
            Gm[l * Ns + m] = acc[q];
            Gm[m * Ns + l] = c64{acc[q].re, -acc[q].im};
        } else if (p < nG + nC) {
            Cm[p - nG] = acc[q];
        } else {
            tn[p - nG - nC] = acc[q].re;
        }
    }
    __syncthreads();
    // Cholesky in place (lower triangle): G = L L^+
    if (threadIdx.x == 0) {
        for (int j = 0; j < Ns; ++j) {
            double d = Gm[j * Ns + j].re;
            for (int k = 0; k < j; ++k)
                d -= Gm[j * Ns + k].re * Gm[j * Ns + k].re + Gm[j * Ns + k].im * Gm[j * Ns + k].im;
            if (!(d > 0.0)) {
                atomicOr(flag, 1);
                d = 1.0;
            }
            const double ljj = sqrt(d);
            Gm[j * Ns + j] = c64{ljj, 0.0};
            for (int i = j + 1; i < Ns; ++i) {
                c64 s = Gm[i * Ns + j];
                for (int k = 0; k < j; ++k) {
                    const c64 a = Gm[i * Ns + k], b = Gm[j * Ns + k];  // s -= L_ik conj(L_jk)
                    s.re -= a.re * b.re + a.im * b.im;
                    s.im -= a.im * b.re - a.re * b.im;
                }
                Gm[i * Ns + j] = c64{s.re / ljj, s.im / ljj};
            }
        }
    }
    __syncthreads();
    // columns of Y: L z = c, L^+ y = z
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        c64 z[kMaxLossN];
        for (int i = 0; i < Ns; ++i) {
            c64 s = Cm[i * K + k];
            for (int j = 0; j < i; ++j) {
                const c64 a = Gm[i * Ns + j];
                s.re -= a.re * z[j].re - a.im * z[j].im;
                s.im -= a.re * z[j].im + a.im * z[j].re;
            }
            const double d = Gm[i * Ns + i].re;
            z[i] = c64{s.re / d, s.im / d};
        }
        for (int i = Ns - 1; i >= 0; --i) {
            c64 s = z[i];
            for (int j = i + 1; j < Ns; ++j) {
                const c64 a = Gm[j * Ns + i];  // (L^+)_ij = conj(L_ji)
                s.re -= a.re * z[j].re + a.im * z[j].im;
                s.im -= a.re * z[j].im - a.im * z[j].re;
            }
            const double d = Gm[i * Ns + i].re;
            z[i] = c64{s.re / d, s.im / d};
        }
        double pr = 0.0;
        for (int i = 0; i < Ns; ++i) {
            const c64 cc = Cm[i * K + k];
            pr += cc.re * z[i].re + cc.im * z[i].im;
            Y[((long)blk * Ns + i) * K + k] = z[i];
        }
        tb2[(long)blk * K + k] = tn[k];
        proj[(long)blk * K + k] = pr;
    }
}

// grad_l(x) = -sum_k (t_k(x) - sum_m Psi_m(x) Y_mk) conj(Y_lk) wk[k]
// (wk = 1 / (K ||t_k||^2)). Workgroup = kLT entries of one block: first the
// residuals r_k(x) into LDS (task (k, x)), then the gradient (task (l, x)).
__global__ __launch_bounds__(256) void k_deficit_grad(Geom g, const c64* __restrict__ Psi, int Ns,
                                                      const c64* __restrict__ T, int K, const c64* __restrict__ Y,
                                                      const double* __restrict__ wk, c64* __restrict__ grad)
{
    __shared__ c64 ys[kMaxLossN * kMaxLossN];
    __shared__ c64 rs[kMaxLossN * kLT];
    __shared__ double ws[kMaxLossN];
    const int blk = blockIdx.y;
    const long F = 12 * g.V;
    const int ne = 12 * g.Vb;
    const int e0 = blockIdx.x * kLT;
    for (int q = threadIdx.x; q < Ns * K; q += blockDim.x)
        ys[q] = Y[(long)blk * Ns * K + q];
    for (int q = threadIdx.x; q < K; q += blockDim.x)
        ws[q] = wk[q];
    __syncthreads();
    auto index = [&](int e) -> long {
        if ((g.Vb & (kTile - 1)) == 0)
            return (long)blk * ne + e;
        return tidx((long)blk * g.Vb + e % g.Vb, e / g.Vb, 12);
    };
    for (int q = threadIdx.x; q < K * kLT; q += blockDim.x) {
        const int k = q / kLT, e = q % kLT;
        c64 r{0.0, 0.0};
        if (e0 + e < ne) {
            const long idx = index(e0 + e);
            r = T[(long)k * F + idx];
            for (int m = 0; m < Ns; ++m) {
                const c64 p = Psi[(long)m * F + idx], y = ys[m * K + k];
                r.re -= p.re * y.re - p.im * y.im;
                r.im -= p.re * y.im + p.im * y.re;
            }
        }
        rs[k * kLT + e] = r;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < Ns * kLT; q += blockDim.x) {
        const int l = q / kLT, e = q % kLT;
        if (e0 + e >= ne)
            continue;
        double gr = 0.0, gi = 0.0;
        for (int k = 0; k < K; ++k) {
            const c64 r = rs[k * kLT + e], y = ys[l * K + k];  // r conj(y)
            gr -= ws[k] * (r.re * y.re + r.im * y.im);
            gi -= ws[k] * (r.im * y.re - r.re * y.im);
        }
        grad[(long)l * F + index(e0 + e)] = c64{gr, gi};
    }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, const float* __restrict__ gr,
                                              float* __restrict__ m, float* __restrict__ v, long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

Lat make_lat(const Geom& g)
{
    Lat lt;
    for (int mu = 0; mu < 4; ++mu)
        lt.L[mu] = g.L[mu];
    lt.str[3] = 1;
    for (int mu = 2; mu >= 0; --mu)
        lt.str[mu] = lt.str[mu + 1] * lt.L[mu + 1];
    lt.V = g.V;
    return lt;
}

inline unsigned site_blocks(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t conv_wgrad_chunk_floats(const Geom& g, int cin, int cout, long* chunk, int* nchunk)
{
    // about 64 workgroups' worth of sites per chunk, at most 32 chunks
    long c = (g.V + 31) / 32;
    c = ((c + kWS - 1) / kWS) * kWS;
    if (c < 4096)
        c = 4096;
    *chunk = c;
    *nchunk = (int)((g.V + c - 1) / c);
    return (size_t)(*nchunk) * 81 * cin * cout;
}

// ------------------------------------- allocation-free weight gradient
//
// Partial sums of the weight gradient for callers that cannot allocate
// (conv4d_backward_noalloc): a file-scope device array of kNoAllocFloats
// floats, which every device the library runs on holds until the process
// ends. Host code takes its device address from hipGetSymbolAddress, once per
// device, and passes that to the kernels (the array's name is no device
// address on the host). Every call overwrites the part it uses before reading
// it; calls that overlap on one device race on it.
static __device__ __align__(256) float scratch[kNoAllocFloats];

float* noalloc_scratch()
{
    static std::mutex mu;
    static float* ptr[kMaxDevices] = {};
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        fail(DFL_EINVAL, "device index beyond the allocation-free scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            fail(DFL_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        ptr[dev] = static_cast<float*>(p);
    }
    return ptr[dev];
}

bool conv_wgrad_chunk_fit(const Geom& g, int cin, int cout, size_t cap, long* chunk, int* nchunk)
{
    const size_t per = (size_t)81 * cin * cout;
    if (conv_wgrad_chunk_floats(g, cin, cout, chunk, nchunk) <= cap)
        return true;
    const long most = (long)(cap / per);
    if (most < 1)
        return false;
    long c = (g.V + most - 1) / most;
    c = ((c + kWS - 1) / kWS) * kWS;
    *chunk = c;
    *nchunk = (int)((g.V + c - 1) / c);
    return (size_t)(*nchunk) * per <= cap;
}

void launch_net_features(const Geom& g, const c64* U64, const float* noise, float* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_features, dim3(site_blocks(g.V)), dim3(256), 0, s, g, U64, noise, x);
}

void launch_conv_forward(const Geom& g, const float* in, int cin, const float* W, const float* b, int cout, float* z,
                         float* a, hipStream_t s)
{
    const Lat lt = make_lat(g);
    if (g.L[3] % 32 == 0)
        hipLaunchKernelGGL(k_conv_mfma<false>, dim3((unsigned)(g.V / 32), (cout + 31) / 32), dim3(256), 0, s, lt, in,
                           cin, W, cin, cout, b, cout, z, a, nullptr);
    else
        hipLaunchKernelGGL(k_conv<false>, dim3(site_blocks(g.V), (cout + kCO - 1) / kCO), dim3(256), 0, s, lt, in,
                           cin, W, cin, cout, b, cout, z, a, nullptr);
}

bool conv_bf16_fits(const Geom& g) { return g.L[3] % kBTS == 0 && g.L[2] % kBNL == 0; }

size_t conv_bf16_weight_elems(int cin, int cout)
{
    const int ot = cout <= 32 ? 2 : 4;
    const int cinP = (cin + kBK - 1) / kBK * kBK, coutP = (cout + 16 * ot - 1) / (16 * ot) * (16 * ot);
    return 81ul * (size_t)cinP * (size_t)coutP;
}

void launch_conv_forward_bf16(const Geom& g, const float* in, int cin, const float* W, const float* b, int cout,
                              float* z, float* a, uint16_t* Wb, hipStream_t s)
{
    const Lat lt = make_lat(g);
    const int ot = cout <= 32 ? 2 : 4;
    const int cinP = (cin + kBK - 1) / kBK * kBK, coutP = (cout + 16 * ot - 1) / (16 * ot) * (16 * ot);
    const long nw = 81L * cinP * coutP;
    hipLaunchKernelGGL(k_weights_bf16, dim3(site_blocks(nw)), dim3(256), 0, s, W, cin, cout, cinP, coutP, Wb);
    const unsigned ngrp = (unsigned)(g.V / (kBTS * kBNL));
    if (ot == 2)
        hipLaunchKernelGGL(k_conv_bf16<2>, dim3(ngrp * (unsigned)(coutP / 32)), dim3(256), 0, s, lt, in, cin, cinP,
                           Wb, coutP, b, cout, z, a);
    else
        hipLaunchKernelGGL(k_conv_bf16<4>, dim3(ngrp * (unsigned)(coutP / 64)), dim3(256), 0, s, lt, in, cin, cinP,
                           Wb, coutP, b, cout, z, a);
}

void launch_conv_backward(const Geom& g, const float* in, int cin, const float* W, int cout, const float* gr,
                          float* dW, float* db, float* din, const float* zprev, float* part, long chunk, int nchunk,
                          hipStream_t s)
{
    const Lat lt = make_lat(g);
    hipLaunchKernelGGL(k_conv_wgrad, dim3(81, (cout + kWT - 1) / kWT, nchunk), dim3(256), 0, s, lt, in, cin, gr,
                       cout, chunk, part);
    const long n = 81L * cin * cout;
    hipLaunchKernelGGL(k_sum_chunks, dim3(site_blocks(n)), dim3(256), 0, s, part, n, nchunk, dW);
    hipLaunchKernelGGL(k_bias_grad, dim3(cout), dim3(256), 0, s, gr, g.V, db);
    if (!din)
        return;
    if (g.L[3] % 32 == 0)
        hipLaunchKernelGGL(k_conv_mfma<true>, dim3((unsigned)(g.V / 32), (cin + 31) / 32), dim3(256), 0, s, lt, gr,
                           cout, W, cin, cout, nullptr, cin, din, nullptr, zprev);
    else
        hipLaunchKernelGGL(k_conv<true>, dim3(site_blocks(g.V), (cin + kCO - 1) / kCO), dim3(256), 0, s, lt, gr,
                           cout, W, cin, cout, nullptr, cin, din, nullptr, zprev);
}

void launch_out_to_fields(const Geom& g, const float* out, int Ns, c64* f, hipStream_t s)
{
    hipLaunchKernelGGL(k_out_to_fields, dim3(site_blocks(g.V)), dim3(256), 0, s, g, out, Ns, f);
}

void launch_fields_to_out(const Geom& g, const c64* gr, int Ns, float* dout, hipStream_t s)
{
    hipLaunchKernelGGL(k_fields_to_out, dim3(site_blocks(g.V)), dim3(256), 0, s, g, gr, Ns, dout);
}

size_t deficit_lds_bytes(int Ns, int K)
{
    return sizeof(c64) * ((size_t)(Ns + K) * (kLT + 1) + (size_t)Ns * Ns + (size_t)Ns * K) + sizeof(double) * K;
}

void launch_deficit_block(const Geom& g, const c64* Psi, int Ns, const c64* T, int K, c64* Y, double* tb2,
                          double* proj, int* flag, hipStream_t s)
{
    const size_t lds = deficit_lds_bytes(Ns, K);
    static std::once_flag attr;
    set_max_lds_once(attr, reinterpret_cast<const void*>(&k_deficit_block), (int)deficit_lds_bytes(kMaxLossN, kMaxLossN));
    hipLaunchKernelGGL(k_deficit_block, dim3(g.Nb), dim3(256), lds, s, g, Psi, Ns, T, K, Y, tb2, proj, flag);
}

void launch_deficit_grad(const Geom& g, const c64* Psi, int Ns, const c64* T, int K, const c64* Y, const double* wk,
                         c64* grad, hipStream_t s)
{
    const int ne = 12 * (int)g.Vb;
    hipLaunchKernelGGL(k_deficit_grad, dim3((ne + kLT - 1) / kLT, g.Nb), dim3(256), 0, s, g, Psi, Ns, T, K, Y, wk,
                       grad);
}

void launch_adam(float* th, const float* gr, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_adam, dim3(site_blocks(n)), dim3(256), 0, s, th, gr, m, v, n, lr, b1, b2, eps, c1, c2);
}

}  // namespace dfl
