// Learned warm start for the gradient flow (a project addition, not in the paper): a small FP32
// MLP maps the physical parameters of a field, (ln beta, gamma_0, gamma_1[, gamma_2]), to its ground
// state on a coarse grid of the same box; the prediction is resampled to the plan's grid by
// band-limited (periodic Dirichlet) interpolation along each axis and normalised, and serves as the
// initial guess of the flow of Sec. 3.1.
// Everything -- forward, backward, loss, Adam -- runs in the kernels below.
//
// Network: x (n_in) -> tanh(W1 x + b1) (H) -> tanh(W2 . + b2) (H) -> W3 . + b3 (n_out).
// Inputs are standardised with the mean / standard deviation of the training inputs.
// Loss: mean squared error over all outputs of a batch.
// Parameter layout (flattened, row-major, in this order): W1 [n_in][H], b1 [H], W2 [H][H], b2 [H],
// W3 [H][n_out], b3 [n_out].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "nlf_internal.h"

struct nlf_model {
    int n_in, H, n_out;
    hipStream_t stream;
    long long np;                 // parameter count
    float* params = nullptr;      // device
    float* grad = nullptr;        // device, same layout
    float* m1 = nullptr;          // Adam moments
    float* m2 = nullptr;
    float* xs = nullptr;          // standardised inputs of the current batch [B][n_in]
    float* a1 = nullptr;          // activations [B][H]
    float* a2 = nullptr;
    float* y = nullptr;           // outputs [B][n_out]
    float* d1 = nullptr;          // backward scratch [B][H]
    float* d2 = nullptr;
    double* lpart = nullptr;      // loss partials
    float* norm = nullptr;        // device: input mean [8], standard deviation [8]
    float* feat = nullptr;        // device: features of up to kMaxFields fields (nlf_ws_predict)
    int* ndev = nullptr;          // device: grid sizes of the plan being predicted for (unused)
    double* rmat = nullptr;       // device: resampling matrices, one per axis [3][nout * nin]
    void* guess[2] = {nullptr, nullptr};   // [batch][n] plan-precision initial guesses (warm start)
    long long guess_cap = 0;      // bytes of each
    double* tmp[2] = {nullptr, nullptr};
    long long tmp_cap = 0;        // elements of each tmp buffer
    int cap_batch = 0;            // rows the scratch buffers hold
    float mean[8], stdv[8];       // input standardisation
    long long adam_t = 0;
    std::vector<void*> owned;
};

namespace nlf {

constexpr int kMaxFields = 8192;

static int ws_alloc(nlf_model* m, void** p, size_t bytes) {
    *p = nullptr;
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(NLF_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    m->owned.push_back(*p);
    return NLF_OK;
}

static long long off_b1(const nlf_model* m) { return (long long)m->n_in * m->H; }
static long long off_W2(const nlf_model* m) { return off_b1(m) + m->H; }
static long long off_b2(const nlf_model* m) { return off_W2(m) + (long long)m->H * m->H; }
static long long off_W3(const nlf_model* m) { return off_b2(m) + m->H; }
static long long off_b3(const nlf_model* m) { return off_W3(m) + (long long)m->H * m->n_out; }

// ---- FP32 GEMM: C[M][N] = op(A) op(B) (+ C if accumulate); op(A) is M x K, op(B) is K x N ----------
// A is [M][K] (TA = 0) or [K][M] (TA = 1); B is [K][N] (TB = 0) or [N][K] (TB = 1); row-major.
// 64 x 64 output tile per workgroup, K staged through LDS in steps of 16, 4 x 4 outputs per thread.
template <int TA, int TB>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* __restrict__ A,
                                              const float* __restrict__ B, float* __restrict__ C, int accumulate) {
    __shared__ float As[16][64 + 4];
    __shared__ float Bs[16][64 + 4];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int idx = threadIdx.x; idx < 16 * 64; idx += 256) {
            int kk = idx / 64, mm = idx % 64;
            int r = row0 + mm, k = k0 + kk;
            float va = 0.f;
            if (r < M && k < K) va = TA ? A[(long long)k * M + r] : A[(long long)r * K + k];
            As[kk][mm] = va;
            int c = col0 + mm;
            float vb = 0.f;
            if (c < N && k < K) vb = TB ? B[(long long)c * K + k] : B[(long long)k * N + c];
            Bs[kk][mm] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int r = row0 + ty * 4 + i;
        if (r >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int c = col0 + tx * 4 + j;
            if (c >= N) continue;
            long long o = (long long)r * N + c;
            C[o] = accumulate ? C[o] + acc[i][j] : acc[i][j];
        }
    }
}

// Z += bias (per column), optionally tanh
__global__ void k_bias_act(int rows, int cols, float* Z, const float* __restrict__ bias, int act) {
    long long n = (long long)rows * cols;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        float v = Z[i] + bias[i % cols];
        Z[i] = act ? tanhf(v) : v;
    }
}

// standardise inputs
__global__ void k_standardise(int rows, int cols, const float* __restrict__ x, float* __restrict__ xs,
                              const float* __restrict__ mean, const float* __restrict__ stdv) {
    long long n = (long long)rows * cols;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        int c = (int)(i % cols);
        xs[i] = (x[i] - mean[c]) / stdv[c];
    }
}

// dY = 2 (Y - T) / count (written over Y); loss partials in FP64
__global__ void k_mse(long long n, float* __restrict__ Y, const float* __restrict__ T, double scale,
                      double* __restrict__ part) {
    double s = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        double d = (double)Y[i] - (double)T[i];
        s += d * d;
        Y[i] = (float)(2.0 * d * scale);
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] * scale;
}

// column sums of D [rows][cols] into g (bias gradients)
__global__ void k_colsum(int rows, int cols, const float* __restrict__ D, float* __restrict__ g) {
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += D[(long long)r * cols + c];
    g[c] = s;
}

// D *= (1 - A^2)   (derivative of tanh at its output A)
__global__ void k_tanh_back(long long n, float* __restrict__ D, const float* __restrict__ A) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        D[i] *= (1.f - A[i] * A[i]);
}

// Adam (Kingma & Ba) with bias correction
__global__ void k_adam(long long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        float gi = g[i];
        float mi = b1 * m[i] + (1.f - b1) * gi;
        float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Band-limited (spectral) resampling along one axis: in [A][nin][C] -> out [A][nout][C],
// out[a][i][c] = sum_j R[i][j] in[a][j][c], R the periodic Dirichlet interpolation matrix.
template <typename TI, typename TO>
__global__ void k_resample_axis(long long A, int nin, int nout, long long C, const TI* __restrict__ in,
                                TO* __restrict__ out, const double* __restrict__ R, int absval) {
    const long long total = A * nout * C;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        long long c = t % C;
        long long r = t / C;
        int i = (int)(r % nout);
        long long a = r / nout;
        const TI* src = in + (a * nin) * C + c;
        const double* row = R + (long long)i * nin;
        double s = 0;
        for (int j = 0; j < nin; ++j) s += row[j] * (double)src[(long long)j * C];
        out[t] = (TO)(absval ? fabs(s) : s);
    }
}

static dim3 grid1(long long n) { return dim3((unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4096))); }

template <int TA, int TB>
static int gemm(nlf_model* m, int M, int N, int K, const float* A, const float* B, float* C, int acc) {
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, m->stream, M, N, K, A, B, C, acc);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

static int ensure_batch(nlf_model* m, int B) {
    if (B <= m->cap_batch) return NLF_OK;
    // scratch grows (old buffers stay owned until destroy)
    NLF_TRY(ws_alloc(m, (void**)&m->xs, (size_t)B * m->n_in * sizeof(float)));
    NLF_TRY(ws_alloc(m, (void**)&m->a1, (size_t)B * m->H * sizeof(float)));
    NLF_TRY(ws_alloc(m, (void**)&m->a2, (size_t)B * m->H * sizeof(float)));
    NLF_TRY(ws_alloc(m, (void**)&m->d1, (size_t)B * m->H * sizeof(float)));
    NLF_TRY(ws_alloc(m, (void**)&m->d2, (size_t)B * m->H * sizeof(float)));
    NLF_TRY(ws_alloc(m, (void**)&m->y, (size_t)B * m->n_out * sizeof(float)));
    m->cap_batch = B;
    return NLF_OK;
}

static int forward(nlf_model* m, int B, const float* x) {
    NLF_TRY(ensure_batch(m, B));
    float* P = m->params;
    hipLaunchKernelGGL(k_standardise, grid1((long long)B * m->n_in), dim3(256), 0, m->stream, B, m->n_in, x, m->xs,
                       m->norm, m->norm + 8);
    NLF_TRY((gemm<0, 0>(m, B, m->H, m->n_in, m->xs, P, m->a1, 0)));
    hipLaunchKernelGGL(k_bias_act, grid1((long long)B * m->H), dim3(256), 0, m->stream, B, m->H, m->a1, P + off_b1(m), 1);
    NLF_TRY((gemm<0, 0>(m, B, m->H, m->H, m->a1, P + off_W2(m), m->a2, 0)));
    hipLaunchKernelGGL(k_bias_act, grid1((long long)B * m->H), dim3(256), 0, m->stream, B, m->H, m->a2, P + off_b2(m), 1);
    NLF_TRY((gemm<0, 0>(m, B, m->n_out, m->H, m->a2, P + off_W3(m), m->y, 0)));
    hipLaunchKernelGGL(k_bias_act, grid1((long long)B * m->n_out), dim3(256), 0, m->stream, B, m->n_out, m->y,
                       P + off_b3(m), 0);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

// loss and gradient (into m->grad) of one batch; loss read back if loss != NULL
static int loss_grad(nlf_model* m, int B, const float* x, const float* t, double* loss) {
    NLF_TRY(forward(m, B, x));
    const long long ny = (long long)B * m->n_out;
    const int nblk = (int)std::min<long long>((ny + 255) / 256, 1024);
    hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, m->stream, ny, m->y, t, 1.0 / (double)ny, m->lpart);
    float* P = m->params;
    float* G = m->grad;
    // layer 3: dW3 = a2^T dY, db3 = colsum dY, d2 = dY W3^T
    NLF_TRY((gemm<1, 0>(m, m->H, m->n_out, B, m->a2, m->y, G + off_W3(m), 0)));
    hipLaunchKernelGGL(k_colsum, dim3((m->n_out + 255) / 256), dim3(256), 0, m->stream, B, m->n_out, m->y, G + off_b3(m));
    NLF_TRY((gemm<0, 1>(m, B, m->H, m->n_out, m->y, P + off_W3(m), m->d2, 0)));
    hipLaunchKernelGGL(k_tanh_back, grid1((long long)B * m->H), dim3(256), 0, m->stream, (long long)B * m->H, m->d2, m->a2);
    // layer 2
    NLF_TRY((gemm<1, 0>(m, m->H, m->H, B, m->a1, m->d2, G + off_W2(m), 0)));
    hipLaunchKernelGGL(k_colsum, dim3((m->H + 255) / 256), dim3(256), 0, m->stream, B, m->H, m->d2, G + off_b2(m));
    NLF_TRY((gemm<0, 1>(m, B, m->H, m->H, m->d2, P + off_W2(m), m->d1, 0)));
    hipLaunchKernelGGL(k_tanh_back, grid1((long long)B * m->H), dim3(256), 0, m->stream, (long long)B * m->H, m->d1, m->a1);
    // layer 1
    NLF_TRY((gemm<1, 0>(m, m->n_in, m->H, B, m->xs, m->d1, G, 0)));
    hipLaunchKernelGGL(k_colsum, dim3((m->H + 255) / 256), dim3(256), 0, m->stream, B, m->H, m->d1, G + off_b1(m));
    NLF_HIP(hipGetLastError());
    if (loss) {
        std::vector<double> h(nblk);
        NLF_HIP(hipMemcpyAsync(h.data(), m->lpart, nblk * sizeof(double), hipMemcpyDeviceToHost, m->stream));
        NLF_HIP(hipStreamSynchronize(m->stream));
        double s = 0;
        for (double v : h) s += v;
        *loss = s;
    }
    return NLF_OK;
}

}  // namespace nlf

using namespace nlf;

extern "C" {

int nlf_ws_create(int n_in, int n_hidden, int n_out, unsigned long long seed, void* stream, nlf_model** out) {
    clear_error();
    if (!out || n_in < 1 || n_in > 8 || n_hidden < 1 || n_out < 1)
        return set_error(NLF_EINVAL, "need 1 <= n_in <= 8, n_hidden >= 1, n_out >= 1 and out != NULL");
    *out = nullptr;
    nlf_model* m = new (std::nothrow) nlf_model();
    if (!m) return set_error(NLF_ENOMEM, "host allocation failed");
    m->n_in = n_in;
    m->H = n_hidden;
    m->n_out = n_out;
    m->stream = (hipStream_t)stream;
    m->np = off_b3(m) + n_out;
    for (int i = 0; i < 8; ++i) { m->mean[i] = 0.f; m->stdv[i] = 1.f; }
    int st = NLF_OK;
    st = st ? st : ws_alloc(m, (void**)&m->params, m->np * sizeof(float));
    st = st ? st : ws_alloc(m, (void**)&m->grad, m->np * sizeof(float));
    st = st ? st : ws_alloc(m, (void**)&m->m1, m->np * sizeof(float));
    st = st ? st : ws_alloc(m, (void**)&m->m2, m->np * sizeof(float));
    st = st ? st : ws_alloc(m, (void**)&m->lpart, 1024 * sizeof(double));
    st = st ? st : ws_alloc(m, (void**)&m->norm, 16 * sizeof(float));
    st = st ? st : ws_alloc(m, (void**)&m->feat, (size_t)kMaxFields * 8 * sizeof(float));
    st = st ? st : ws_alloc(m, (void**)&m->ndev, 3 * sizeof(int));
    st = st ? st : ws_alloc(m, (void**)&m->rmat, (size_t)3 * 1024 * 1024 * sizeof(double));
    if (st == NLF_OK) {
        // Glorot-uniform weights, zero biases (host-side deterministic init from the seed)
        std::vector<float> p(m->np, 0.f);
        std::mt19937_64 rng(seed);
        auto fill = [&](long long off, int fan_in, int fan_out) {
            float a = std::sqrt(6.f / (fan_in + fan_out));
            std::uniform_real_distribution<float> u(-a, a);
            for (long long i = 0; i < (long long)fan_in * fan_out; ++i) p[off + i] = u(rng);
        };
        fill(0, n_in, n_hidden);
        fill(off_W2(m), n_hidden, n_hidden);
        fill(off_W3(m), n_hidden, n_out);
        // copies and fills on the model's stream (which may be non-blocking), completed before return
        float ms[16];
        for (int i = 0; i < 8; ++i) { ms[i] = m->mean[i]; ms[8 + i] = m->stdv[i]; }
        if (hipMemcpyAsync(m->params, p.data(), m->np * sizeof(float), hipMemcpyHostToDevice, m->stream) != hipSuccess ||
            hipMemsetAsync(m->m1, 0, m->np * sizeof(float), m->stream) != hipSuccess ||
            hipMemsetAsync(m->m2, 0, m->np * sizeof(float), m->stream) != hipSuccess ||
            hipMemcpyAsync(m->norm, ms, sizeof ms, hipMemcpyHostToDevice, m->stream) != hipSuccess ||
            hipStreamSynchronize(m->stream) != hipSuccess)
            st = set_error(NLF_EHIP, "initialising the model failed");
    }
    if (st != NLF_OK) {
        for (void* q : m->owned) (void)hipFree(q);
        delete m;
        return st;
    }
    *out = m;
    return NLF_OK;
}

int nlf_ws_destroy(nlf_model* m) {
    clear_error();
    if (!m) return NLF_OK;
    (void)hipStreamSynchronize(m->stream);
    for (void* q : m->owned) (void)hipFree(q);
    delete m;
    return NLF_OK;
}

int nlf_ws_num_params(const nlf_model* m, long long* count) {
    clear_error();
    if (!m || !count) return set_error(NLF_EINVAL, "model and count must not be NULL");
    *count = m->np;
    return NLF_OK;
}

int nlf_ws_params(nlf_model* m, float* host_out, const float* host_in) {
    clear_error();
    if (!m) return set_error(NLF_EINVAL, "model must not be NULL");
    // ordered with the model's own work on its stream (which may be non-blocking)
    if (host_in) NLF_HIP(hipMemcpyAsync(m->params, host_in, m->np * sizeof(float), hipMemcpyHostToDevice, m->stream));
    if (host_out) NLF_HIP(hipMemcpyAsync(host_out, m->params, m->np * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    NLF_HIP(hipStreamSynchronize(m->stream));
    return NLF_OK;
}

int nlf_ws_set_standardisation(nlf_model* m, const float* mean, const float* stdv) {
    clear_error();
    if (!m || !mean || !stdv) return set_error(NLF_EINVAL, "model, mean and stdv must not be NULL");
    float ms[16];
    for (int i = 0; i < 8; ++i) {
        ms[i] = (i < m->n_in) ? mean[i] : 0.f;
        ms[8 + i] = (i < m->n_in) ? stdv[i] : 1.f;
        if (i < m->n_in && !(ms[8 + i] > 0.f)) return set_error(NLF_EINVAL, "stdv must be positive");
        m->mean[i] = ms[i];
        m->stdv[i] = ms[8 + i];
    }
    NLF_HIP(hipMemcpyAsync(m->norm, ms, sizeof ms, hipMemcpyHostToDevice, m->stream));
    NLF_HIP(hipStreamSynchronize(m->stream));
    return NLF_OK;
}

int nlf_ws_forward(nlf_model* m, int batch, const float* x, float* y) {
    clear_error();
    if (!m || !x || !y || batch < 1) return set_error(NLF_EINVAL, "model, x, y must not be NULL; batch >= 1");
    NLF_TRY(forward(m, batch, x));
    NLF_HIP(hipMemcpyAsync(y, m->y, (size_t)batch * m->n_out * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
    return NLF_OK;
}

int nlf_ws_loss_grad(nlf_model* m, int batch, const float* x, const float* t, float* grad, double* loss) {
    clear_error();
    if (!m || !x || !t || batch < 1) return set_error(NLF_EINVAL, "model, x, t must not be NULL; batch >= 1");
    NLF_TRY(loss_grad(m, batch, x, t, loss));
    if (grad) NLF_HIP(hipMemcpyAsync(grad, m->grad, m->np * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
    NLF_HIP(hipStreamSynchronize(m->stream));
    return NLF_OK;
}

int nlf_ws_train(nlf_model* m, int n, const float* x, const float* t, int epochs, int minibatch, double lr,
                 double* loss_host) {
    clear_error();
    if (!m || !x || !t || n < 1 || epochs < 0) return set_error(NLF_EINVAL, "bad arguments to nlf_ws_train");
    const int mb = (minibatch > 0 && minibatch < n) ? minibatch : n;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int e = 0; e < epochs; ++e) {
        double esum = 0;
        int nb = 0;
        for (int s = 0; s < n; s += mb) {
            int B = std::min(mb, n - s);
            double l = 0;
            const bool want = loss_host != nullptr;
            NLF_TRY(loss_grad(m, B, x + (long long)s * m->n_in, t + (long long)s * m->n_out, want ? &l : nullptr));
            ++m->adam_t;
            float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
            hipLaunchKernelGGL(k_adam, grid1(m->np), dim3(256), 0, m->stream, m->np, m->params, m->grad, m->m1, m->m2,
                               (float)lr, b1, b2, eps, c1, c2);
            NLF_HIP(hipGetLastError());
            esum += l;
            ++nb;
        }
        if (loss_host) loss_host[e] = esum / nb;
    }
    NLF_HIP(hipStreamSynchronize(m->stream));
    return NLF_OK;
}

int nlf_ws_predict(nlf_model* m, nlf_plan* p, const nlf_phys* phys, int coarse_n, void* psi0) {
    clear_error();
    if (!m || !p || !phys || !psi0 || coarse_n < 2) return set_error(NLF_EINVAL, "bad arguments to nlf_ws_predict");
    const int B = p->batch;
    if (B > kMaxFields) return set_error(NLF_EINVAL, "at most %d fields per prediction", kMaxFields);
    long long ncd = 1;
    for (int a = 0; a < p->dim; ++a) ncd *= coarse_n;
    if (m->n_out != ncd) return set_error(NLF_EINVAL, "model output %d != coarse_n^dim = %lld", m->n_out, ncd);
    if (m->n_in != 1 + p->dim) return set_error(NLF_EINVAL, "model input must be 1 + dim features");
    std::vector<float> feat((size_t)B * m->n_in);
    for (int b = 0; b < B; ++b) {
        if (!(phys[b].beta > 0)) return set_error(NLF_EINVAL, "warm start needs beta > 0");
        feat[(size_t)b * m->n_in] = (float)std::log(phys[b].beta);
        for (int a = 0; a < p->dim; ++a) feat[(size_t)b * m->n_in + 1 + a] = (float)phys[b].gamma[a];
    }
    float* fx = m->feat;
    NLF_HIP(hipMemcpyAsync(fx, feat.data(), feat.size() * sizeof(float), hipMemcpyHostToDevice, m->stream));
    NLF_TRY(forward(m, B, fx));
    // band-limited interpolation matrices, coarse (nc points) -> fine (n_a points) on the same box:
    // R[i][j] = D(2 pi (i/n_a - j/nc)), D(t) = (1 + 2 sum_{k=1}^{nc/2-1} cos(k t) + cos(nc t / 2)) / nc
    const int nc = coarse_n;
    if (nc % 2 || nc > 1024) return set_error(NLF_EINVAL, "coarse_n must be even and <= 1024");
    std::vector<double> R;
    for (int a = 0; a < p->dim; ++a) {
        const int nf = p->n[a];
        if ((long long)nf * nc > 1024 * 1024) return set_error(NLF_EINVAL, "resampling matrix too large");
        for (int i = 0; i < nf; ++i)
            for (int j = 0; j < nc; ++j) {
                long double t = 2.0L * 3.141592653589793238462643383279502884L * ((long double)i / nf - (long double)j / nc);
                long double v = 1.0L + cosl(0.5L * nc * t);
                for (int k = 1; k < nc / 2; ++k) v += 2.0L * cosl(k * t);
                R.push_back((double)(v / nc));
            }
    }
    NLF_HIP(hipMemcpyAsync(m->rmat, R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice, m->stream));
    // axis by axis, last axis first: [B][nc..][nc] -> ... -> [B][n0]..[n_{d-1}]
    long long need = (long long)B;
    for (int a = 0; a < p->dim; ++a) need *= std::max(nc, p->n[a]);
    if (need > m->tmp_cap) {
        NLF_TRY(ws_alloc(m, (void**)&m->tmp[0], need * sizeof(double)));
        NLF_TRY(ws_alloc(m, (void**)&m->tmp[1], need * sizeof(double)));
        m->tmp_cap = need;
    }
    int dims[3];
    for (int a = 0; a < p->dim; ++a) dims[a] = nc;
    const double* roff[3];
    {
        long long o = 0;
        for (int a = 0; a < p->dim; ++a) { roff[a] = m->rmat + o; o += (long long)p->n[a] * nc; }
    }
    const void* src = m->y;
    bool src_float = true;
    int cur = 0;
    for (int a = p->dim - 1; a >= 0; --a) {
        long long A = B, C = 1;
        for (int q = 0; q < a; ++q) A *= dims[q];
        for (int q = a + 1; q < p->dim; ++q) C *= dims[q];
        const long long total = A * p->n[a] * C;
        const bool last = (a == 0);
        const dim3 g((unsigned)std::min<long long>((total + 255) / 256, 8192));
        if (last && p->prec == NLF_F32) {
            if (src_float)
                hipLaunchKernelGGL((k_resample_axis<float, float>), g, dim3(256), 0, m->stream, A, nc, p->n[a], C,
                                   (const float*)src, (float*)psi0, roff[a], 1);
            else
                hipLaunchKernelGGL((k_resample_axis<double, float>), g, dim3(256), 0, m->stream, A, nc, p->n[a], C,
                                   (const double*)src, (float*)psi0, roff[a], 1);
        } else {
            double* dst = last ? (double*)psi0 : m->tmp[cur];
            if (src_float)
                hipLaunchKernelGGL((k_resample_axis<float, double>), g, dim3(256), 0, m->stream, A, nc, p->n[a], C,
                                   (const float*)src, dst, roff[a], last ? 1 : 0);
            else
                hipLaunchKernelGGL((k_resample_axis<double, double>), g, dim3(256), 0, m->stream, A, nc, p->n[a], C,
                                   (const double*)src, dst, roff[a], last ? 1 : 0);
            src = dst;
            src_float = false;
            cur ^= 1;
        }
        NLF_HIP(hipGetLastError());
        dims[a] = p->n[a];
    }
    NLF_HIP(hipStreamSynchronize(m->stream));
    return NLF_OK;
}

int nlf_ws_ground_state(nlf_model* m, int coarse_n, nlf_plan* p, const nlf_phys* phys, const nlf_gf_opts* gf,
                        void* psi, nlf_gs_stats* stats, int* used) {
    clear_error();
    if (!m || !p || !phys || !psi || !stats) return set_error(NLF_EINVAL, "bad arguments to nlf_ws_ground_state");
    const int B = p->batch;
    const long long bytes = (long long)B * p->N * (long long)(elem_size(p->prec) / 2);
    if (bytes > m->guess_cap) {
        NLF_TRY(ws_alloc(m, &m->guess[0], bytes));
        NLF_TRY(ws_alloc(m, &m->guess[1], bytes));
        m->guess_cap = bytes;
    }
    // the network's guess and the harmonic-oscillator Gaussian
    NLF_TRY(nlf_ws_predict(m, p, phys, coarse_n, m->guess[0]));
    NLF_TRY(ho_guess(p, phys, m->guess[1]));
    // judge: residual of one gradient-flow step from each start (the output buffer is scratch here)
    nlf_gf_opts one = gf ? *gf : nlf_gf_opts{};
    one.max_iter = 1;
    one.mixed = 0;
    std::vector<nlf_gs_stats> sw(B), sg(B);
    int st = nlf_ground_state(p, phys, &one, m->guess[0], psi, sw.data());
    if (st != NLF_OK && st != NLF_ENOCONV) return st;
    st = nlf_ground_state(p, phys, &one, m->guess[1], psi, sg.data());
    if (st != NLF_OK && st != NLF_ENOCONV) return st;
    // per field: keep the network's guess only where its residual is smaller
    const size_t es = elem_size(p->prec) / 2;
    for (int b = 0; b < B; ++b) {
        const bool warm = sw[b].residual < sg[b].residual;
        if (used) used[b] = warm ? 1 : 0;
        if (!warm)
            NLF_HIP(hipMemcpyAsync((char*)m->guess[0] + (size_t)b * p->N * es, (char*)m->guess[1] + (size_t)b * p->N * es,
                                   p->N * es, hipMemcpyDeviceToDevice, p->stream));
    }
    st = nlf_ground_state(p, phys, gf, m->guess[0], psi, stats);
    if (st == NLF_OK || st == NLF_ENOCONV)
        for (int b = 0; b < B; ++b) stats[b].iters += 2;   // the two judging steps
    return st;
}

}  // extern "C"
