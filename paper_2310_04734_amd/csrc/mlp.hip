// Learned expansion-point proposer: a small MLP trained on the GPU by the library's own
// forward and backward kernels.
//
//   input  x: n_in features (log10 candidate residuals, max-subtracted, then geometry features)
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3)      (hidden width H)
//   logits = W4 h3 + b4                                                     (n_out candidates)
//   loss = mean over the batch of -log softmax(logits masked to allowed classes)[label]
//
// Weights are held as FP32 master copies and used in BF16 (rounded to nearest even) by the
// forward and backward products, which run on the matrix cores (BF16 MFMA, FP32 accumulation);
// Adam updates the FP32 masters and re-rounds the BF16 copies. Activations and gradients stay
// FP32 and enter the products as two BF16 parts (hi + lo), so they keep 16 significant bits.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "util.cuh"

namespace cr {
namespace {

__device__ __forceinline__ float bf16_round(float x) {
    // round to nearest even on the top 16 bits (NaN kept quiet)
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;
    unsigned lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    return __uint_as_float(u);
}

constexpr int kT = 16;   // MFMA tile (16 x 16 outputs per wave, K = 16 per instruction)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) { return (short)(__float_as_uint(bf16_round(x)) >> 16); }
__device__ __forceinline__ float bf16_value(short b) { return __uint_as_float(((unsigned)(unsigned short)b) << 16); }

// C[m, n] (+)= sum_k A[m, k] B[k, n] with arbitrary strides on the matrix cores
// (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation); optional bias[n], relu, and relu' mask from Z
// (C *= (Z > 0)). An FP32 operand is split into bf16 hi + lo parts (hi = bf16(x), lo = bf16(x - hi),
// 16 significant bits together) and multiplied part by part: hi*hi + lo*hi (SPLIT_A) + hi*lo
// (SPLIT_B); an operand that is already bf16-valued (the weights) is not split. Operand layout of
// the instruction on gfx950: A[i][k] in lane i + 16 (k / 4), item k % 4; B[k][j] in lane
// j + 16 (k / 4), item k % 4; output item r of lane l is D[4 (l / 16) + r][l % 16].
// 256 threads = 4 waves, each one 16 x 16 tile of a 32 x 32 block.
template <bool SPLIT_A, bool SPLIT_B>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* __restrict__ A, int64_t sam, int64_t sak,
                                              const float* __restrict__ B, int64_t sbk, int64_t sbn, float* __restrict__ Cm,
                                              int64_t scm, int64_t scn, const float* __restrict__ bias, int relu,
                                              const float* __restrict__ Z, int64_t szm, int64_t szn, int accumulate) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 32 + 16 * (w & 1), n0 = blockIdx.x * 32 + 16 * (w >> 1);
    const int ia = m0 + (lane & 15), jb = n0 + (lane & 15), kq = 4 * (lane >> 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += kT) {
        bf16x4 ah, al, bh, bl;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = k0 + kq + e;
            const float av = (ia < M && k < K) ? A[ia * sam + k * sak] : 0.f;
            const float bv = (k < K && jb < N) ? B[k * sbk + jb * sbn] : 0.f;
            ah[e] = bf16_bits(av);
            bh[e] = bf16_bits(bv);
            if (SPLIT_A) al[e] = bf16_bits(av - bf16_value(ah[e]));
            if (SPLIT_B) bl[e] = bf16_bits(bv - bf16_value(bh[e]));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
        if (SPLIT_A) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
        if (SPLIT_B) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    }
    const int n = n0 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = m0 + 4 * (lane >> 4) + r;
        if (m < M && n < N) {
            float v = acc[r];
            if (bias) v += bias[n];
            if (accumulate) v += Cm[m * scm + n * scn];
            if (relu) v = fmaxf(v, 0.f);
            if (Z && !(Z[m * szm + n * szn] > 0.f)) v = 0.f;
            Cm[m * scm + n * scn] = v;
        }
    }
}

// per sample: masked softmax, loss, and dlogits = (p - onehot) / batch
__global__ void k_softmax_ce(int batch, int n_out, const float* __restrict__ logits, const int32_t* __restrict__ labels,
                             const float* __restrict__ mask, float* __restrict__ dlogits, float* __restrict__ loss) {
    const int b = blockIdx.x;
    if (b >= batch) return;
    __shared__ float red[256];
    const float* z = logits + (size_t)b * n_out;
    float mx = -INFINITY;
    for (int j = threadIdx.x; j < n_out; j += blockDim.x)
        if (!mask || mask[(size_t)b * n_out + j] > 0.f) mx = fmaxf(mx, z[j]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    mx = red[0];
    __syncthreads();
    float sum = 0.f;
    for (int j = threadIdx.x; j < n_out; j += blockDim.x)
        if (!mask || mask[(size_t)b * n_out + j] > 0.f) sum += expf(z[j] - mx);
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    sum = red[0];
    const int lab = labels[b];
    for (int j = threadIdx.x; j < n_out; j += blockDim.x) {
        const bool ok = !mask || mask[(size_t)b * n_out + j] > 0.f;
        const float p = ok ? expf(z[j] - mx) / sum : 0.f;
        dlogits[(size_t)b * n_out + j] = (p - (j == lab ? 1.f : 0.f)) / (float)batch;
    }
    if (threadIdx.x == 0) loss[b] = -(z[lab] - mx - logf(sum));
}

// db[n] = sum_m G[m, n]
__global__ void k_colsum(int M, int N, const float* __restrict__ G, float* __restrict__ db) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += G[(size_t)m * N + n];
    db[n] = s;
}

__global__ void k_adam(int64_t n, float* __restrict__ w, float* __restrict__ wb, const float* __restrict__ g,
                       float* __restrict__ m1, float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float mh = a / c1, vh = b / c2;
    w[i] -= lr * mh / (sqrtf(vh) + eps);
    wb[i] = bf16_round(w[i]);
}

__global__ void k_round_bf16(int64_t n, const float* __restrict__ w, float* __restrict__ wb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = bf16_round(w[i]);
}

}  // namespace
}  // namespace cr

using namespace cr;

struct cr_mlp_s {
    cr_ctx ctx = nullptr;
    int n_in = 0, H = 0, n_out = 0;
    int64_t np = 0;
    int64_t off[8] = {0};   // W1 b1 W2 b2 W3 b3 W4 b4
    int64_t sz[8] = {0};
    DevBuf<float> w, wb, g, m1, m2;   // master, bf16-rounded copy, gradient, Adam moments
    int64_t step = 0;
    DevBuf<float> act, dact, logits, dlog, loss, xin;
    DevBuf<int32_t> lab;
    int cap = 0;
};

namespace {

void layout(cr_mlp m) {
    const int64_t dims[4][2] = {{m->H, m->n_in}, {m->H, m->H}, {m->H, m->H}, {m->n_out, m->H}};
    int64_t o = 0;
    for (int l = 0; l < 4; ++l) {
        m->off[2 * l] = o;
        m->sz[2 * l] = dims[l][0] * dims[l][1];
        o += m->sz[2 * l];
        m->off[2 * l + 1] = o;
        m->sz[2 * l + 1] = dims[l][0];
        o += dims[l][0];
    }
    m->np = o;
}

void reserve_batch(cr_mlp m, int batch) {
    if (batch <= m->cap) return;
    m->act.alloc((size_t)batch * m->H * 6);    // z1 a1 z2 a2 z3 a3 (z kept for relu')
    m->dact.alloc((size_t)batch * m->H * 2);
    m->logits.alloc((size_t)batch * m->n_out);
    m->dlog.alloc((size_t)batch * m->n_out);
    m->loss.alloc(batch);
    m->cap = batch;
}

// operand kinds: the weights are bf16-valued (used as they are), activations and gradients are
// FP32 (split into bf16 hi + lo)
enum { kF32 = 0, kBF16 = 1 };

void gemm(hipStream_t s, int M, int N, int K, const float* A, int64_t sam, int64_t sak, int kind_a, const float* B,
          int64_t sbk, int64_t sbn, int kind_b, float* Cm, int64_t scm, int64_t scn, const float* bias, int relu,
          const float* Z = nullptr, int64_t szm = 0, int64_t szn = 0) {
    dim3 grid((N + 31) / 32, (M + 31) / 32);
    const bool sa = kind_a == kF32, sb = kind_b == kF32;
    if (sa && sb)
        hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, Cm, scm, scn,
                           bias, relu, Z, szm, szn, 0);
    else if (sa)
        hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, Cm, scm, scn,
                           bias, relu, Z, szm, szn, 0);
    else if (sb)
        hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, Cm, scm, scn,
                           bias, relu, Z, szm, szn, 0);
    else
        hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, Cm, scm, scn,
                           bias, relu, Z, szm, szn, 0);
}

// forward on X (batch x n_in): activations z_l (pre-relu), a_l, logits
void forward(cr_mlp m, int batch, const float* X) {
    hipStream_t s = m->ctx->stream;
    reserve_batch(m, batch);
    const int H = m->H;
    float* z[3];
    float* a[3];
    for (int l = 0; l < 3; ++l) {
        z[l] = m->act.p + (size_t)batch * H * (2 * l);
        a[l] = m->act.p + (size_t)batch * H * (2 * l + 1);
    }
    const float* Wb = m->wb.p;
    const float* w = m->w.p;
    // z = a_prev W^T + b  : C[b, o] = sum_i A[b, i] W[o, i]
    const float* in = X;
    int nin = m->n_in;
    for (int l = 0; l < 3; ++l) {
        gemm(s, batch, H, nin, in, nin, 1, kF32, Wb + m->off[2 * l], 1, nin, kBF16, z[l], H, 1, w + m->off[2 * l + 1], 0);
        gemm(s, batch, H, nin, in, nin, 1, kF32, Wb + m->off[2 * l], 1, nin, kBF16, a[l], H, 1, w + m->off[2 * l + 1], 1);
        in = a[l];
        nin = H;
    }
    gemm(s, batch, m->n_out, H, a[2], H, 1, kF32, Wb + m->off[6], 1, H, kBF16, m->logits.p, m->n_out, 1, w + m->off[7], 0);
}

float backward(cr_mlp m, int batch, const float* X, const int32_t* labels, const float* mask) {
    hipStream_t s = m->ctx->stream;
    const int H = m->H, no = m->n_out;
    hipLaunchKernelGGL(k_softmax_ce, dim3(batch), dim3(256), 0, s, batch, no, m->logits.p, labels, mask, m->dlog.p,
                       m->loss.p);
    float* z[3];
    float* a[3];
    for (int l = 0; l < 3; ++l) {
        z[l] = m->act.p + (size_t)batch * H * (2 * l);
        a[l] = m->act.p + (size_t)batch * H * (2 * l + 1);
    }
    float* g = m->g.p;
    const float* Wb = m->wb.p;
    // layer 4: dW4[o, i] = sum_b dlog[b, o] a3[b, i]; db4 = colsum(dlog); da3 = dlog W4 (masked by z3 > 0)
    float* d_cur = m->dact.p;
    float* d_nxt = m->dact.p + (size_t)batch * H;
    gemm(s, no, H, batch, m->dlog.p, 1, no, kF32, a[2], H, 1, kF32, g + m->off[6], H, 1, nullptr, 0);
    hipLaunchKernelGGL(k_colsum, dim3((no + 255) / 256), dim3(256), 0, s, batch, no, m->dlog.p, g + m->off[7]);
    gemm(s, batch, H, no, m->dlog.p, no, 1, kF32, Wb + m->off[6], H, 1, kBF16, d_cur, H, 1, nullptr, 0, z[2], H, 1);
    for (int l = 2; l >= 0; --l) {
        const float* in = l > 0 ? a[l - 1] : X;
        const int nin = l > 0 ? H : m->n_in;
        gemm(s, H, nin, batch, d_cur, 1, H, kF32, in, nin, 1, kF32, g + m->off[2 * l], nin, 1, nullptr, 0);
        hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, batch, H, d_cur, g + m->off[2 * l + 1]);
        if (l > 0) {
            gemm(s, batch, H, H, d_cur, H, 1, kF32, Wb + m->off[2 * l], H, 1, kBF16, d_nxt, H, 1, nullptr, 0, z[l - 1], H, 1);
            std::swap(d_cur, d_nxt);
        }
    }
    std::vector<float> hl(batch);
    CR_HIP(hipMemcpyAsync(hl.data(), m->loss.p, batch * sizeof(float), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    double tot = 0;
    for (float v : hl) tot += v;
    return (float)(tot / batch);
}

}  // namespace

namespace cr {
// network input: log10 residuals shifted so that the largest is 0, then the geometry features;
// mask: 0 at used candidates and their neighbours, 1 elsewhere
void mlp_features(int nc, const double* res, int n_used, const int* used, int ng, const double* geom, float* x,
                  float* mask) {
    double mx = -1e300;
    for (int c = 0; c < nc; ++c) mx = std::max(mx, std::log10(std::max(res[c], 1e-300)));
    for (int c = 0; c < nc; ++c) x[c] = (float)(std::log10(std::max(res[c], 1e-300)) - mx);
    for (int k = 0; k < ng; ++k) x[nc + k] = geom ? (float)geom[k] : 0.f;
    if (mask) {
        for (int c = 0; c < nc; ++c) mask[c] = 1.f;
        for (int k = 0; k < n_used; ++k)
            for (int d = -1; d <= 1; ++d)
                if (used[k] + d >= 0 && used[k] + d < nc) mask[used[k] + d] = 0.f;
    }
}

int mlp_propose(cr_mlp m, const std::vector<double>& res, const std::vector<int>& used, const double* geom) {
    const int nc = (int)res.size();
    const int ng = m->n_in - m->n_out;
    if (nc != m->n_out || ng < 0) throw Error(CR_E_INVALID, "network does not match the candidate count");
    std::vector<float> x(m->n_in, 0.f), mask(nc);
    mlp_features(nc, res.data(), (int)used.size(), used.data(), ng, geom, x.data(), mask.data());
    hipStream_t s = m->ctx->stream;
    m->xin.reserve(m->n_in);
    CR_HIP(hipMemcpyAsync(m->xin.p, x.data(), m->n_in * sizeof(float), hipMemcpyHostToDevice, s));
    forward(m, 1, m->xin.p);
    std::vector<float> lg(nc);
    CR_HIP(hipMemcpyAsync(lg.data(), m->logits.p, nc * sizeof(float), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    int best = -1;
    for (int c = 0; c < nc; ++c) {
        if (mask[c] == 0.f) continue;
        if (best < 0 || lg[c] > lg[best]) best = c;
    }
    return best;
}
}  // namespace cr

extern "C" {

cr_status cr_mlp_features(int32_t n_cand, const double* res, int32_t n_used, const int32_t* used, int32_t n_geom,
                          const double* geom, float* x, float* mask) {
    if (n_cand < 1 || !res || !x || n_used < 0 || (n_used > 0 && !used) || n_geom < 0 || (n_geom > 0 && !geom))
        return CR_E_INVALID;
    cr::mlp_features(n_cand, res, n_used, used, n_geom, geom, x, mask);
    return CR_OK;
}

cr_status cr_mlp_create(cr_ctx ctx, int32_t n_in, int32_t hidden, int32_t n_out, uint64_t seed, cr_mlp* out) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(out && n_in > 0 && hidden > 0 && n_out > 0 && n_in <= 65536 && hidden <= 8192 && n_out <= 65536,
                   CR_E_INVALID, "cr_mlp_create: bad sizes");
        auto m = std::make_unique<cr_mlp_s>();
        m->ctx = ctx;
        m->n_in = n_in;
        m->H = hidden;
        m->n_out = n_out;
        layout(m.get());
        // He-uniform initialisation from SplitMix64 (weights), zero biases
        std::vector<float> h(m->np, 0.f);
        uint64_t st = seed;
        auto next = [&]() {
            st += 0x9E3779B97F4A7C15ull;
            uint64_t z = st;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            return (double)(z >> 11) * (1.0 / 9007199254740992.0);
        };
        const int fan_in[4] = {n_in, hidden, hidden, hidden};
        for (int l = 0; l < 4; ++l) {
            const double a = std::sqrt(6.0 / fan_in[l]);
            for (int64_t i = 0; i < m->sz[2 * l]; ++i) h[m->off[2 * l] + i] = (float)((2 * next() - 1) * a);
        }
        hipStream_t s = ctx->stream;
        m->w.alloc(m->np);
        m->wb.alloc(m->np);
        m->g.alloc(m->np);
        m->m1.alloc(m->np);
        m->m2.alloc(m->np);
        CR_HIP(hipMemcpyAsync(m->w.p, h.data(), m->np * sizeof(float), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_round_bf16, dim3((unsigned)((m->np + 255) / 256)), dim3(256), 0, s, m->np, m->w.p, m->wb.p);
        fill_zero(m->m1.p, m->np, s);
        fill_zero(m->m2.p, m->np, s);
        fill_zero(m->g.p, m->np, s);
        CR_HIP(hipStreamSynchronize(s));
        *out = m.release();
    });
}

void cr_mlp_destroy(cr_mlp m) { delete m; }

cr_status cr_mlp_forward(cr_mlp m, int32_t batch, const float* X_dev, float* logits_dev) {
    if (!m) return CR_E_INVALID;
    return cr_guard(m->ctx, [&] {
        CR_REQUIRE(batch > 0 && X_dev && logits_dev, CR_E_INVALID, "cr_mlp_forward: bad arguments");
        forward(m, batch, X_dev);
        CR_HIP(hipMemcpyAsync(logits_dev, m->logits.p, (size_t)batch * m->n_out * sizeof(float), hipMemcpyDeviceToDevice,
                              m->ctx->stream));
        CR_HIP(hipStreamSynchronize(m->ctx->stream));
    });
}

cr_status cr_mlp_gradients(cr_mlp m, int32_t batch, const float* X_dev, const int32_t* labels_dev, const float* mask_dev,
                           float* grad_dev, float* loss_out) {
    if (!m) return CR_E_INVALID;
    return cr_guard(m->ctx, [&] {
        CR_REQUIRE(batch > 0 && X_dev && labels_dev, CR_E_INVALID, "cr_mlp_gradients: bad arguments");
        forward(m, batch, X_dev);
        const float l = backward(m, batch, X_dev, labels_dev, mask_dev);
        if (loss_out) *loss_out = l;
        if (grad_dev)
            CR_HIP(hipMemcpyAsync(grad_dev, m->g.p, m->np * sizeof(float), hipMemcpyDeviceToDevice, m->ctx->stream));
        CR_HIP(hipStreamSynchronize(m->ctx->stream));
    });
}

cr_status cr_mlp_train_step(cr_mlp m, int32_t batch, const float* X_dev, const int32_t* labels_dev, const float* mask_dev,
                            float lr, float* loss_out) {
    if (!m) return CR_E_INVALID;
    return cr_guard(m->ctx, [&] {
        CR_REQUIRE(batch > 0 && X_dev && labels_dev && lr > 0, CR_E_INVALID, "cr_mlp_train_step: bad arguments");
        forward(m, batch, X_dev);
        const float l = backward(m, batch, X_dev, labels_dev, mask_dev);
        m->step++;
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((m->np + 255) / 256)), dim3(256), 0, m->ctx->stream, m->np, m->w.p,
                           m->wb.p, m->g.p, m->m1.p, m->m2.p, lr, b1, b2, eps, c1, c2);
        CR_HIP(hipStreamSynchronize(m->ctx->stream));
        if (loss_out) *loss_out = l;
    });
}

cr_status cr_mlp_num_params(cr_mlp m, int64_t* n) {
    if (!m || !n) return CR_E_INVALID;
    *n = m->np;
    return CR_OK;
}

cr_status cr_mlp_get_params(cr_mlp m, float* params) {
    if (!m) return CR_E_INVALID;
    return cr_guard(m->ctx, [&] {
        CR_REQUIRE(params, CR_E_INVALID, "cr_mlp_get_params: null output");
        CR_HIP(hipMemcpyAsync(params, m->w.p, m->np * sizeof(float), hipMemcpyDeviceToHost, m->ctx->stream));
        CR_HIP(hipStreamSynchronize(m->ctx->stream));
    });
}

cr_status cr_mlp_set_params(cr_mlp m, const float* params) {
    if (!m) return CR_E_INVALID;
    return cr_guard(m->ctx, [&] {
        CR_REQUIRE(params, CR_E_INVALID, "cr_mlp_set_params: null input");
        hipStream_t s = m->ctx->stream;
        CR_HIP(hipMemcpyAsync(m->w.p, params, m->np * sizeof(float), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_round_bf16, dim3((unsigned)((m->np + 255) / 256)), dim3(256), 0, s, m->np, m->w.p, m->wb.p);
        CR_HIP(hipStreamSynchronize(s));
    });
}

}  // extern "C"
