// nc_guide.hip -- the learned proposal: an MLP from a scattering vertex
// (normalised position, incoming direction, log extinction) to a mixture of
// von Mises-Fisher lobes over the outgoing direction, trained on the
// tracer's own vertices by weighted maximum likelihood.
//
// Network 15 -> 64 -> 64 -> 64 -> 40 (8 lobes x (logit, mean direction 3,
// log concentration)), ReLU on hidden layers; its inputs are a vertex's 7
// values and 8 Fourier features of its horizontal position (guide_feature).  Products run on the matrix
// cores (v_mfma_f32_16x16x16_bf16: bf16 operands, fp32 accumulation); master
// weights, Adam moments and gradients are fp32.  Padded layer shapes (in x
// out): 16x64, 64x64, 64x64, 64x48.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "nc_internal.hpp"

namespace nc {

// ---------------------------------------------------------------------------
// Shapes and parameter layout (flat fp32, per layer W [out][in] row-major
// then b [out]; the same order as the oracle's)
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int guide_in(int l) { return l == 0 ? kGuideIn : kGuideWidth; }
__host__ __device__ constexpr int guide_out(int l) { return l == kGuideLayers - 1 ? kGuideOut : kGuideWidth; }
__host__ __device__ constexpr int guide_in_pad(int l) { return l == 0 ? 16 : kGuideWidth; }
__host__ __device__ constexpr int guide_out_pad(int l) { return l == kGuideLayers - 1 ? 48 : kGuideWidth; }

// ---------------------------------------------------------------------------
// Matrix-core fragments.  For v_mfma_f32_16x16x16_bf16, lane l (0..63) holds
//   A[m][k] for m = l % 16, k = 4 (l / 16) + i  (i = 0..3),
//   B[k][n] for n = l % 16, k = 4 (l / 16) + i,
//   D[m][n] for n = l % 16, m = 4 (l / 16) + i.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Forward over tiles of 16 records.  One wave per block; the tile's hidden
// activations go through LDS between layers.  X: records as rows of
// `rec_stride` floats, the vertex's 7 values first (the 15 network inputs
// are formed from them).  Outputs: Z (n x 48, fp32, before
// any activation of the last layer) and, for training, the hidden
// activations H_l (n x 64, fp32, after ReLU) of layers 0..2.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void guide_forward_kernel(GuideWeights W, const float *__restrict__ X, int n,
                                                           int rec_stride, float *__restrict__ Z,
                                                           float *__restrict__ H0, float *__restrict__ H1,
                                                           float *__restrict__ H2)
{
    __shared__ float act[16][kGuideWidth + 4];
    const int l = threadIdx.x;
    const int mrow = l & 15, kq = l >> 4;
    float *Hs[3] = {H0, H1, H2};
    for (int tile = blockIdx.x; tile * 16 < n; tile += gridDim.x) {
        const int r0 = tile * 16;
        // inputs into the activation buffer (columns 0..15, zero padded)
        for (int e = l; e < 16 * 16; e += 64) {
            const int m = e >> 4, k = e & 15;
            const int r = r0 + m;
            act[m][k] = (r < n && k < kGuideIn) ? guide_feature(X + (size_t)r * rec_stride, k) : 0.0f;
        }
        __syncthreads();
        for (int layer = 0; layer < kGuideLayers; ++layer) {
            const int kin = guide_in_pad(layer), nout = guide_out_pad(layer);
            f32x4 acc[4];
            for (int nt = 0; nt < nout / 16; ++nt) {
                f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
                for (int kt = 0; kt < kin / 16; ++kt) {
                    bf16x4 a, b;
                    const int kk = kt * 16 + 4 * kq;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        a[i] = to_bf16(act[mrow][kk + i]);
                        b[i] = W.w[layer][(size_t)(nt * 16 + mrow) * kin + kk + i];
                    }
                    c = mfma16(a, b, c);
                }
                acc[nt] = c;
            }
            __syncthreads();   // all lanes have read act
            for (int nt = 0; nt < nout / 16; ++nt) {
                const int ncol = nt * 16 + mrow;
                const float bias = W.b[layer][ncol];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = 4 * kq + i;
                    float v = acc[nt][i] + bias;
                    const int r = r0 + m;
                    if (layer < kGuideLayers - 1) {
                        v = fmaxf(v, 0.0f);
                        act[m][ncol] = v;
                        if (Hs[layer] && r < n) Hs[layer][(size_t)r * kGuideWidth + ncol] = v;
                    } else if (r < n) {
                        Z[(size_t)r * 48 + ncol] = v;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Mixture of vMF lobes from the raw outputs of one record.
// ---------------------------------------------------------------------------
__device__ inline float vmf_norm(float kappa)
{
    // kappa / (2 pi (1 - exp(-2 kappa)))
    return kappa / (2.0f * kPi * (-expm1f(-2.0f * kappa)));
}

// Loss terms and d loss / d outputs for records with weight w:
//   L = -sum w ln q / sum w, q = sum_j pi_j vmf(mu_j, kappa_j; w_out).
__global__ void guide_loss_kernel(const float *__restrict__ Z, const float *__restrict__ rec, int n, int rec_stride,
                                  const double *__restrict__ wsum, float *__restrict__ dZ, double *__restrict__ loss)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    double li = 0.0;
    if (r < n) {
        const float *z = Z + (size_t)r * 48;
        const float *q = rec + (size_t)r * rec_stride;
        const float wo[3] = {q[7], q[8], q[9]};
        const float wr = q[10];
        const float inv_w = (float)(1.0 / wsum[0]);
        float amax = z[0];
        for (int j = 1; j < kGuideLobes; ++j) amax = fmaxf(amax, z[5 * j]);
        float pi[kGuideLobes], v[kGuideLobes], kap[kGuideLobes], cw[kGuideLobes], nm[kGuideLobes];
        float mu[kGuideLobes][3];
        float psum = 0.0f;
        for (int j = 0; j < kGuideLobes; ++j) {
            pi[j] = expf(z[5 * j] - amax);
            psum += pi[j];
        }
        float qv = 0.0f;
        for (int j = 0; j < kGuideLobes; ++j) {
            pi[j] /= psum;
            const float m0 = z[5 * j + 1], m1 = z[5 * j + 2], m2 = z[5 * j + 3];
            nm[j] = fmaxf(sqrtf(m0 * m0 + m1 * m1 + m2 * m2), 1e-12f);
            mu[j][0] = m0 / nm[j];
            mu[j][1] = m1 / nm[j];
            mu[j][2] = m2 / nm[j];
            kap[j] = expf(fminf(fmaxf(z[5 * j + 4], kLogKappaMin), kLogKappaMax));
            cw[j] = mu[j][0] * wo[0] + mu[j][1] * wo[1] + mu[j][2] * wo[2];
            v[j] = vmf_norm(kap[j]) * expf(kap[j] * (cw[j] - 1.0f));
            qv += pi[j] * v[j];
        }
        qv = fmaxf(qv, 1e-30f);
        li = -(double)wr * log((double)qv);
        float *g = dZ + (size_t)r * 48;
        const float s = -wr * inv_w;
        for (int j = 0; j < kGuideLobes; ++j) {
            const float rj = pi[j] * v[j] / qv;
            g[5 * j] = s * (rj - pi[j]);
            const float e2 = expf(-2.0f * kap[j]);
            const float dlk = 1.0f / kap[j] - 2.0f * e2 / (-expm1f(-2.0f * kap[j])) + (cw[j] - 1.0f);
            const float zs = z[5 * j + 4];
            g[5 * j + 4] = (zs > kLogKappaMin && zs < kLogKappaMax) ? s * rj * dlk * kap[j] : 0.0f;
            const float f = s * rj * kap[j] / nm[j];
            for (int a = 0; a < 3; ++a) g[5 * j + 1 + a] = f * (wo[a] - cw[j] * mu[j][a]);
        }
        for (int c = kGuideOut; c < 48; ++c) g[c] = 0.0f;
    }
    // block reduction of the loss
    __shared__ double red[256];
    red[threadIdx.x] = li;
    __syncthreads();
    for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) unsafeAtomicAdd(loss, red[0]);
}

__global__ void weight_sum_kernel(const float *__restrict__ rec, int n, int rec_stride, double *out)
{
    double s = 0.0;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        s += (double)rec[(size_t)r * rec_stride + 10];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) unsafeAtomicAdd(out, red[0]);
}

// ---------------------------------------------------------------------------
// The whole backward pass over one chunk of records per workgroup (4 waves).
// Each tile of 16 records is staged in LDS once (the last layer's output
// gradient, the hidden activations H0..H2 and the network inputs, as fp32
// columns [unit][record]); then, from the last layer to the first, the
// weight gradient dW_l += dZ_l^T Hin_l (the records are the product's k) and,
// for l > 0, dZ_{l-1} = (dZ_l W_l) masked by the ReLU of H_{l-1}, both on the
// matrix cores.  A wave keeps its share of the weight-gradient tiles in
// registers over the whole chunk: layer 3 tiles (o-tile 0..2, i-tile = wave),
// layers 2 and 1 (o-tile 0..3, i-tile = wave), layer 0 (o-tile = wave); the
// bias sums ride on the A fragments of the waves with i-tile 0.  At the end
// every parameter's sum is written once to the workgroup's row of `part`
// (no atomics; the Adam kernel adds the rows).
// ---------------------------------------------------------------------------
constexpr int kColPad = 20;   // floats per LDS column of 16 records (16 + 4 keeps float4 alignment)

__host__ __device__ constexpr int guide_param_off(int l)
{
    return l == 0 ? 0 : guide_param_off(l - 1) + guide_out(l - 1) * guide_in(l - 1) + guide_out(l - 1);
}
static_assert(guide_param_off(kGuideLayers) == kGuideParams, "parameter layout");

__device__ inline bf16x4 col_frag(const float *col, int kq, float *sum)
{
    const float4 v = *reinterpret_cast<const float4 *>(col + 4 * kq);
    if (sum) *sum += (v.x + v.y) + (v.z + v.w);
    bf16x4 a;
    a[0] = to_bf16(v.x);
    a[1] = to_bf16(v.y);
    a[2] = to_bf16(v.z);
    a[3] = to_bf16(v.w);
    return a;
}

__global__ __launch_bounds__(256) void guide_backward_kernel(GuideWeights W, const float *__restrict__ rec,
                                                             int rec_stride, const float *__restrict__ dZ4,
                                                             const float *__restrict__ H0, const float *__restrict__ H1,
                                                             const float *__restrict__ H2, int n, int chunk,
                                                             float *__restrict__ part)
{
    __shared__ __align__(16) float hc[3][kGuideWidth][kColPad];    // H0..H2 by column
    __shared__ __align__(16) float xc[16][kColPad];                 // network inputs by column
    __shared__ __align__(16) float zc[2][kGuideWidth][kColPad];    // dZ by column (current, next layer)
    __shared__ __align__(16) float zr[2][16][kGuideWidth + 4];     // dZ by row
    __shared__ __align__(16) short wts[3][kGuideWidth][kGuideWidth + 8];   // W_l^T [in][out], l = 1..3
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int mrow = lane & 15, kq = lane >> 4;
    for (int L = 1; L < kGuideLayers; ++L) {
        const int op = guide_out_pad(L);
        for (int e = tid; e < kGuideWidth * op; e += 256) wts[L - 1][e / op][e % op] = W.wt[L][e];
    }
    f32x4 g3[3], g2[4], g1[4], g0;
    float b3[3], b2[4], b1[4], b0 = 0.0f;
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t < 3) g3[t] = zero, b3[t] = 0.0f;
        g2[t] = zero, g1[t] = zero, b2[t] = 0.0f, b1[t] = 0.0f;
    }
    g0 = zero;
    const int rbeg = blockIdx.x * chunk, rend = min(n, rbeg + chunk);
    const bool bias_wave = wv == 0;
    for (int r0 = rbeg; r0 < rend; r0 += 16) {
        __syncthreads();   // the previous tile is done with the LDS
        {
            // thread -> record m of the tile, four consecutive columns c4
            const int m = tid >> 4, c4 = (tid & 15) * 4;
            const int r = r0 + m;
            const bool ok = r < rend;
            const float *Hs[3] = {H0, H1, H2};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float4 v = ok ? *reinterpret_cast<const float4 *>(Hs[k] + (size_t)r * kGuideWidth + c4)
                                    : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                hc[k][c4][m] = v.x;
                hc[k][c4 + 1][m] = v.y;
                hc[k][c4 + 2][m] = v.z;
                hc[k][c4 + 3][m] = v.w;
            }
            if (c4 < 48) {
                const float4 v = ok ? *reinterpret_cast<const float4 *>(dZ4 + (size_t)r * 48 + c4)
                                    : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                zc[0][c4][m] = v.x;
                zc[0][c4 + 1][m] = v.y;
                zc[0][c4 + 2][m] = v.z;
                zc[0][c4 + 3][m] = v.w;
                *reinterpret_cast<float4 *>(&zr[0][m][c4]) = v;
            }
            if (c4 < 16) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    xc[c4 + j][m] = (ok && c4 + j < kGuideIn) ? guide_feature(rec + (size_t)r * rec_stride, c4 + j)
                                                              : 0.0f;
            }
        }
        __syncthreads();
        // layer L: weight gradient, then (L > 0) the input gradient into the other buffer
        auto backprop = [&](int L, int cur, int ktiles) {
            f32x4 c = zero;
            const int i = 16 * wv + mrow;
            for (int kt = 0; kt < ktiles; ++kt) {
                const int o = 16 * kt + 4 * kq;
                const float4 v = *reinterpret_cast<const float4 *>(&zr[cur][mrow][o]);
                bf16x4 a;
                a[0] = to_bf16(v.x);
                a[1] = to_bf16(v.y);
                a[2] = to_bf16(v.z);
                a[3] = to_bf16(v.w);
                const bf16x4 b = *reinterpret_cast<const bf16x4 *>(&wts[L - 1][i][o]);
                c = mfma16(a, b, c);
            }
            // lane holds dZ_{L-1}[r = 4 kq + j][i]
            const float4 h = *reinterpret_cast<const float4 *>(&hc[L - 1][i][4 * kq]);
            float4 d;
            d.x = h.x > 0.0f ? c[0] : 0.0f;
            d.y = h.y > 0.0f ? c[1] : 0.0f;
            d.z = h.z > 0.0f ? c[2] : 0.0f;
            d.w = h.w > 0.0f ? c[3] : 0.0f;
            *reinterpret_cast<float4 *>(&zc[cur ^ 1][i][4 * kq]) = d;
            zr[cur ^ 1][4 * kq][i] = d.x;
            zr[cur ^ 1][4 * kq + 1][i] = d.y;
            zr[cur ^ 1][4 * kq + 2][i] = d.z;
            zr[cur ^ 1][4 * kq + 3][i] = d.w;
        };
        {   // layer 3: in H2, out 48 (3 o-tiles)
            const bf16x4 b = col_frag(hc[2][16 * wv + mrow], kq, nullptr);
#pragma unroll
            for (int ot = 0; ot < 3; ++ot)
                g3[ot] = mfma16(col_frag(zc[0][16 * ot + mrow], kq, bias_wave ? &b3[ot] : nullptr), b, g3[ot]);
            backprop(3, 0, 3);
        }
        __syncthreads();
        {   // layer 2: in H1
            const bf16x4 b = col_frag(hc[1][16 * wv + mrow], kq, nullptr);
#pragma unroll
            for (int ot = 0; ot < 4; ++ot)
                g2[ot] = mfma16(col_frag(zc[1][16 * ot + mrow], kq, bias_wave ? &b2[ot] : nullptr), b, g2[ot]);
            backprop(2, 1, 4);
        }
        __syncthreads();
        {   // layer 1: in H0
            const bf16x4 b = col_frag(hc[0][16 * wv + mrow], kq, nullptr);
#pragma unroll
            for (int ot = 0; ot < 4; ++ot)
                g1[ot] = mfma16(col_frag(zc[0][16 * ot + mrow], kq, bias_wave ? &b1[ot] : nullptr), b, g1[ot]);
            backprop(1, 0, 4);
        }
        __syncthreads();
        // layer 0: in the 15 network inputs (one i-tile), o-tile = wave
        g0 = mfma16(col_frag(zc[1][16 * wv + mrow], kq, &b0), col_frag(xc[mrow], kq, nullptr), g0);
    }
    // write the workgroup's sums: weights from the D fragments (o = 16 ot + 4 kq + j,
    // i = 16 it + mrow), biases reduced over the four lane groups (o = 16 ot + mrow)
    float *P = part + (size_t)blockIdx.x * kGuideParams;
    auto put_w = [&](int L, int ot, int it, const f32x4 &acc) {
        const int on = guide_out(L), in_n = guide_in(L), i = 16 * it + mrow;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = 16 * ot + 4 * kq + j;
            if (o < on && i < in_n) P[guide_param_off(L) + o * in_n + i] = acc[j];
        }
    };
    auto put_b = [&](int L, int ot, float bsum) {
        bsum += __shfl_xor(bsum, 16);
        bsum += __shfl_xor(bsum, 32);
        const int o = 16 * ot + mrow;
        if (kq == 0 && o < guide_out(L)) P[guide_param_off(L) + guide_out(L) * guide_in(L) + o] = bsum;
    };
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        if (ot < 3) put_w(3, ot, wv, g3[ot]);
        put_w(2, ot, wv, g2[ot]);
        put_w(1, ot, wv, g1[ot]);
    }
    put_w(0, wv, 0, g0);
    put_b(0, wv, b0);
    if (bias_wave) {
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            if (ot < 3) put_b(3, ot, b3[ot]);
            put_b(2, ot, b2[ot]);
            put_b(1, ot, b1[ot]);
        }
    }
}

// ---------------------------------------------------------------------------
// The gradient as the sum of the workgroups' rows, then (apply) Adam on the
// fp32 master parameter and its bf16 copies in the padded weight matrices
// (padding entries are never written: they stay zero).
// ---------------------------------------------------------------------------
struct GuidePacked {
    short *w[4];
    short *wt[4];
    float *b[4];
};

// Block of 256 threads per 32 parameters: eight groups of 32 threads add
// every eighth row (consecutive parameters: coalesced rows), then LDS.
constexpr int kAdamParams = 32;

__global__ __launch_bounds__(256) void guide_adam_kernel(float *p, float *m, float *v, float *g,
                                                         const float *__restrict__ part, int nparts, int apply,
                                                         float lr, float b1, float b2, float eps, float c1, float c2,
                                                         GuidePacked out)
{
    __shared__ float red[8][kAdamParams];
    const int t = threadIdx.x & (kAdamParams - 1), grp = threadIdx.x / kAdamParams;
    const int q = blockIdx.x * kAdamParams + t;
    float s = 0.0f;
    if (q < kGuideParams)
        for (int k = grp; k < nparts; k += 8) s += part[(size_t)k * kGuideParams + q];
    red[grp][t] = s;
    __syncthreads();
    if (grp != 0 || q >= kGuideParams) return;
    float gi = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) gi += red[k][t];
    g[q] = gi;
    if (!apply) return;
    const float mi = b1 * m[q] + (1.0f - b1) * gi;
    const float vi = b2 * v[q] + (1.0f - b2) * gi * gi;
    m[q] = mi;
    v[q] = vi;
    const float pq = p[q] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[q] = pq;
    int L = 0;
    while (L + 1 < kGuideLayers && q >= guide_param_off(L + 1)) ++L;
    const int e = q - guide_param_off(L), on = guide_out(L), in_n = guide_in(L);
    if (e < on * in_n) {
        const int o = e / in_n, i = e - o * in_n;
        const short h = to_bf16(pq);
        out.w[L][o * guide_in_pad(L) + i] = h;
        out.wt[L][i * guide_out_pad(L) + o] = h;
    } else {
        out.b[L][e - on * in_n] = pq;
    }
}

__global__ void pack_weights_kernel(const float *params, short *w, short *wt, float *bias, int param_off, int out_n,
                                    int in_n, int out_pad, int in_pad)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= out_pad * in_pad) return;
    const int o = e / in_pad, i = e % in_pad;
    const float val = (o < out_n && i < in_n) ? params[param_off + o * in_n + i] : 0.0f;
    const short h = to_bf16(val);
    w[(size_t)o * in_pad + i] = h;
    wt[(size_t)i * out_pad + o] = h;
    if (i == 0) bias[o] = o < out_n ? params[param_off + out_n * in_n + o] : 0.0f;
}

__global__ void fill_f64_kernel(double *p, size_t n, double v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
GuideWeights guide_weights(const nc_guide *gd)
{
    GuideWeights W;
    for (int l = 0; l < kGuideLayers; ++l) {
        W.w[l] = gd->d_w[l];
        W.wt[l] = gd->d_wt[l];
        W.b[l] = gd->d_bias[l];
    }
    return W;
}

hipError_t guide_pack(const nc_ctx *ctx, nc_guide *gd)
{
    for (int l = 0; l < kGuideLayers; ++l) {
        const int op = guide_out_pad(l), ip = guide_in_pad(l);
        hipLaunchKernelGGL(pack_weights_kernel, dim3((op * ip + 255) / 256), dim3(256), 0, ctx->stream, gd->d_params,
                           gd->d_w[l], gd->d_wt[l], gd->d_bias[l], guide_param_off(l), guide_out(l), guide_in(l), op,
                           ip);
    }
    return hipGetLastError();
}

hipError_t guide_forward(const nc_ctx *ctx, const nc_guide *gd, const float *X, int n, int rec_stride, float *Z,
                         float *H0, float *H1, float *H2)
{
    const int tiles = (n + 15) / 16;
    const int blocks = std::max(1, std::min(tiles, 65536));
    hipLaunchKernelGGL(guide_forward_kernel, dim3(blocks), dim3(64), 0, ctx->stream, guide_weights(gd), X, n,
                       rec_stride, Z, H0, H1, H2);
    return hipGetLastError();
}

// Workgroups of the backward pass: chunks of at least 128 records, at most
// kBwdParts of them (their partial gradients are rows of the scratch buffer).
constexpr int kBwdParts = 512;

static void backward_split(int n, int &parts, int &chunk)
{
    parts = std::max(1, std::min(kBwdParts, (n + 127) / 128));
    chunk = (((n + parts - 1) / parts) + 15) & ~15;
    parts = std::max(1, (n + chunk - 1) / chunk);
}

hipError_t guide_ensure_scratch(nc_guide *gd, int n)
{
    if (gd->scratch_cap >= n) return hipSuccess;
    if (gd->d_scratch) (void)hipFree(gd->d_scratch);
    gd->d_scratch = nullptr;
    gd->scratch_cap = 0;
    // Z (48) + dZ4 (48) + H0..H2 (3 x 64) floats per record, then the
    // backward pass's partial gradients (kBwdParts rows of kGuideParams)
    const size_t per = 48 + 48 + 3 * kGuideWidth;
    hipError_t e = hipMalloc(&gd->d_scratch, sizeof(float) * (per * (size_t)n + (size_t)kBwdParts * kGuideParams));
    if (e == hipSuccess) gd->scratch_cap = n;
    return e;
}

hipError_t guide_train_step(const nc_ctx *ctx, nc_guide *gd, const float *rec, int n, int rec_stride, float lr,
                            double *d_loss, bool apply)
{
    hipError_t e = guide_ensure_scratch(gd, n);
    if (e != hipSuccess) return e;
    float *Z = gd->d_scratch;
    float *dZ4 = Z + (size_t)48 * n;
    float *H[3];
    for (int k = 0; k < 3; ++k) H[k] = dZ4 + (size_t)48 * n + (size_t)k * kGuideWidth * n;
    float *part = H[2] + (size_t)kGuideWidth * n;
    // the loss / weight-sum accumulators start at zero
    hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(64), 0, ctx->stream, gd->d_acc, (size_t)2, 0.0);
    hipLaunchKernelGGL(weight_sum_kernel, dim3(std::max(1, std::min(1024, (n + 255) / 256))), dim3(256), 0,
                       ctx->stream, rec, n, rec_stride, gd->d_acc + 1);
    if ((e = guide_forward(ctx, gd, rec, n, rec_stride, Z, H[0], H[1], H[2])) != hipSuccess) return e;
    hipLaunchKernelGGL(guide_loss_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, Z, rec, n, rec_stride,
                       (const double *)(gd->d_acc + 1), dZ4, gd->d_acc);
    int parts = 1, chunk = 16;
    backward_split(n, parts, chunk);
    hipLaunchKernelGGL(guide_backward_kernel, dim3(parts), dim3(256), 0, ctx->stream, guide_weights(gd), rec,
                       rec_stride, (const float *)dZ4, (const float *)H[0], (const float *)H[1], (const float *)H[2],
                       n, chunk, part);
    float c1 = 1.0f, c2 = 1.0f;
    const float b1 = 0.9f, b2 = 0.999f;
    if (apply) {
        gd->step += 1;
        c1 = 1.0f - std::pow(b1, (float)gd->step);
        c2 = 1.0f - std::pow(b2, (float)gd->step);
    }
    GuidePacked out;
    for (int l = 0; l < kGuideLayers; ++l) {
        out.w[l] = gd->d_w[l];
        out.wt[l] = gd->d_wt[l];
        out.b[l] = gd->d_bias[l];
    }
    hipLaunchKernelGGL(guide_adam_kernel, dim3((kGuideParams + kAdamParams - 1) / kAdamParams), dim3(256), 0, ctx->stream, gd->d_params,
                       gd->d_m, gd->d_v, gd->d_grad, (const float *)part, parts, apply ? 1 : 0, lr, b1, b2, 1e-8f,
                       c1, c2, out);
    if (d_loss) {
        e = hipMemcpyAsync(d_loss, gd->d_acc, 2 * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace nc
