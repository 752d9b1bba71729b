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

static int param_offset(int l)
{
    int off = 0;
    for (int k = 0; k < l; ++k) off += guide_out(k) * guide_in(k) + guide_out(k);
    return off;
}

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
// Backward through the hidden layers: dH_{l-1} = (dZ_l W_l) masked by the
// ReLU of H_{l-1}.  dZ_l: n x out_pad; output n x 64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void guide_backprop_kernel(const short *__restrict__ wt, int out_pad,
                                                            const float *__restrict__ dZ, const float *__restrict__ Hprev,
                                                            float *__restrict__ dZprev, int n)
{
    const int l = threadIdx.x;
    const int mrow = l & 15, kq = l >> 4;
    for (int tile = blockIdx.x; tile * 16 < n; tile += gridDim.x) {
        const int r0 = tile * 16;
        for (int nt = 0; nt < kGuideWidth / 16; ++nt) {
            f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int kt = 0; kt < out_pad / 16; ++kt) {
                bf16x4 a, b;
                const int kk = kt * 16 + 4 * kq;
                const int r = r0 + mrow;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    a[i] = to_bf16(r < n ? dZ[(size_t)r * out_pad + kk + i] : 0.0f);
                    b[i] = wt[(size_t)(nt * 16 + mrow) * out_pad + kk + i];   // W^T[in][out] -> B[k=out][n=in]
                }
                c = mfma16(a, b, c);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + 4 * kq + i;
                const int col = nt * 16 + mrow;
                if (r < n) {
                    const float h = Hprev[(size_t)r * kGuideWidth + col];
                    dZprev[(size_t)r * kGuideWidth + col] = h > 0.0f ? c[i] : 0.0f;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradients dW[o][i] += sum_r dZ[r][o] H[r][i] and db[o] += sum_r dZ[r][o]
// over one chunk of records per block (split over the record axis, fp32
// atomics into the gradient).  One wave per (o-tile, i-tile) of the layer.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void guide_wgrad_kernel(const float *__restrict__ dZ, int out_pad, int out_n,
                                                         const float *__restrict__ H, int h_stride, int in_n,
                                                         int in_pad, int n, int chunk, float *__restrict__ gW,
                                                         float *__restrict__ gb, int features)
{
    const int l = threadIdx.x;
    const int mrow = l & 15, kq = l >> 4;
    const int ot = blockIdx.y / (in_pad / 16), it = blockIdx.y % (in_pad / 16);
    const int rbeg = blockIdx.x * chunk, rend = min(n, rbeg + chunk);
    f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    for (int r0 = rbeg; r0 < rend; r0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + 4 * kq + i;
            const bool ok = r < rend;
            const int col = it * 16 + mrow;
            const float dz = ok ? dZ[(size_t)r * out_pad + ot * 16 + mrow] : 0.0f;     // A[m=o][k=r]
            // B[k=r][n=i]: layer 0 reads the records and forms the network inputs
            const float hv = !(ok && col < in_n) ? 0.0f
                             : features ? guide_feature(H + (size_t)r * h_stride, col)
                                        : H[(size_t)r * h_stride + col];
            a[i] = to_bf16(dz);
            b[i] = to_bf16(hv);
            if (it == 0) bsum += dz;
        }
        c = mfma16(a, b, c);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int o = ot * 16 + 4 * kq + i, in = it * 16 + mrow;
        if (o < out_n && in < in_n) unsafeAtomicAdd(gW + (size_t)o * in_n + in, c[i]);
    }
    if (it == 0) {
        // bsum holds this lane's partial over records 4 kq + i of every step, for o = ot*16 + mrow
        bsum += __shfl_xor(bsum, 16);
        bsum += __shfl_xor(bsum, 32);
        const int o = ot * 16 + mrow;
        if (kq == 0 && o < out_n) unsafeAtomicAdd(gb + o, bsum);
    }
}

// ---------------------------------------------------------------------------
// Adam on the fp32 master parameters, then the bf16 copies.
// ---------------------------------------------------------------------------
__global__ void adam_kernel(float *p, float *m, float *v, const float *g, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
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

__global__ void fill_f32_kernel(float *p, size_t n, float v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
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
                           gd->d_w[l], gd->d_wt[l], gd->d_bias[l], param_offset(l), guide_out(l), guide_in(l), op,
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

hipError_t guide_ensure_scratch(nc_guide *gd, int n)
{
    if (gd->scratch_cap >= n) return hipSuccess;
    if (gd->d_scratch) (void)hipFree(gd->d_scratch);
    gd->d_scratch = nullptr;
    gd->scratch_cap = 0;
    // Z (48) + dZ4 (48) + H0..H2 (3 x 64) + dZ3..dZ1 (3 x 64) floats per record
    const size_t per = 48 + 48 + 6 * kGuideWidth;
    hipError_t e = hipMalloc(&gd->d_scratch, per * sizeof(float) * (size_t)n);
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
    float *H[3], *dZh[3];
    for (int k = 0; k < 3; ++k) {
        H[k] = dZ4 + (size_t)48 * n + (size_t)k * kGuideWidth * n;
        dZh[k] = dZ4 + (size_t)48 * n + (size_t)(3 + k) * kGuideWidth * n;
    }
    const int np = kGuideParams;
    // zero the gradient and the loss / weight-sum accumulators
    hipLaunchKernelGGL(fill_f32_kernel, dim3(64), dim3(256), 0, ctx->stream, gd->d_grad, (size_t)np, 0.0f);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(64), 0, ctx->stream, gd->d_acc, (size_t)2, 0.0);
    hipLaunchKernelGGL(weight_sum_kernel, dim3(std::max(1, std::min(1024, (n + 255) / 256))), dim3(256), 0,
                       ctx->stream, rec, n, rec_stride, gd->d_acc + 1);
    if ((e = guide_forward(ctx, gd, rec, n, rec_stride, Z, H[0], H[1], H[2])) != hipSuccess) return e;
    hipLaunchKernelGGL(guide_loss_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, Z, rec, n, rec_stride,
                       (const double *)(gd->d_acc + 1), dZ4, gd->d_acc);
    // backward: layer 3 (out 48 pad), then hidden layers
    const int tiles = std::max(1, std::min((n + 15) / 16, 65536));
    const float *dZ_cur = dZ4;
    int out_pad = 48;
    for (int l = kGuideLayers - 1; l >= 0; --l) {
        const int on = guide_out(l), in_n = guide_in(l), ip = guide_in_pad(l);
        const float *Hin = l == 0 ? rec : H[l - 1];
        const int hstride = l == 0 ? rec_stride : kGuideWidth;
        const int chunk = 1024;
        dim3 grid((n + chunk - 1) / chunk, (guide_out_pad(l) / 16) * (ip / 16));
        float *gW = gd->d_grad + param_offset(l);
        float *gb = gW + (size_t)on * in_n;
        hipLaunchKernelGGL(guide_wgrad_kernel, grid, dim3(64), 0, ctx->stream, dZ_cur, out_pad, on, Hin, hstride,
                           in_n, ip, n, chunk, gW, gb, l == 0 ? 1 : 0);
        if (l > 0) {
            hipLaunchKernelGGL(guide_backprop_kernel, dim3(tiles), dim3(64), 0, ctx->stream,
                               (const short *)gd->d_wt[l], out_pad, dZ_cur, (const float *)H[l - 1], dZh[l - 1], n);
            dZ_cur = dZh[l - 1];
            out_pad = kGuideWidth;
        }
    }
    if (!apply) {
        if (d_loss) e = hipMemcpyAsync(d_loss, gd->d_acc, 2 * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
        return e != hipSuccess ? e : hipGetLastError();
    }
    gd->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)gd->step), c2 = 1.0f - std::pow(b2, (float)gd->step);
    hipLaunchKernelGGL(adam_kernel, dim3((np + 255) / 256), dim3(256), 0, ctx->stream, gd->d_params, gd->d_m, gd->d_v,
                       (const float *)gd->d_grad, np, lr, b1, b2, 1e-8f, c1, c2);
    if ((e = guide_pack(ctx, gd)) != hipSuccess) return e;
    if (d_loss) {
        e = hipMemcpyAsync(d_loss, gd->d_acc, 2 * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace nc
