// kg_mlp.hip -- the blow-up surrogate: an MLP 4 -> H -> H -> 2 (GELU, FP32)
// mapping Gaussian initial-data parameters (A, sx, sy, sz) to a blow-up
// logit and a standardised log blow-up time, with hand-written forward,
// backward and Adam kernels.  Parametric blow-up studies are the paper's
// motivation (Sec. 1); the network is trained on runs of the solver and the
// solver remains the arbiter (low-confidence answers are rerun).
//
// Loss over a batch of B samples with labels y_b (1 = blow-up) and targets
// t_b (used where y_b = 1):
//   L = (1/B) sum BCE(z1_b, y_b) + (1/max(1, sum y_b)) sum y_b (z2_b - t_b)^2,
//   BCE(z, y) = max(z, 0) - z y + log(1 + exp(-|z|)),  GELU(x) = x/2 (1 + erf(x/sqrt2)).
// Every sum runs in a fixed order, so results are bitwise repeatable.  The
// layers are at most 128 wide and a batch is a few hundred samples, so the
// products are small loops per output rather than matrix-core tiles.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/kg.h"

namespace {

constexpr int NIN = 4, NOUT = 2;

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x)
{
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// Input standardisation, passed by value to the kernels.
struct Norm {
    float mean[NIN], stdev[NIN];
};

// xs = (x - mean) / std
__global__ void k_standardize(const float *x, Norm norm, float *xs, int B)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * NIN) return;
    const int c = i % NIN;
    xs[i] = (x[i] - norm.mean[c]) / norm.stdev[c];
}

// z[b][o] = sum_i in[b][i] W[o][i] + bias[o]; a = GELU(z) when act.
__global__ void k_linear_fwd(const float *in, const float *W, const float *bias, float *z, float *a,
                             int B, int I, int O, int act)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * O) return;
    const int b = idx / O, o = idx % O;
    const float *x = in + (long)b * I, *w = W + (long)o * I;
    float s = bias[o];
    for (int i = 0; i < I; ++i) s += x[i] * w[i];
    z[idx] = s;
    if (act) a[idx] = gelu(s);
}

// Loss and dL/dout for one batch (a single workgroup, fixed-order sums).
__global__ __launch_bounds__(256) void k_loss(const float *out, const float *y, float *dout, float *loss,
                                              int B)
{
    __shared__ float red[256];
    float c = 0.0f;
    for (int b = threadIdx.x; b < B; b += 256) c += y[2 * b];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const float cnt = fmaxf(1.0f, red[0]);
    __syncthreads();
    float l = 0.0f;
    for (int b = threadIdx.x; b < B; b += 256) {
        const float z1 = out[2 * b], z2 = out[2 * b + 1];
        const float lab = y[2 * b], tgt = y[2 * b + 1];
        const float sig = 1.0f / (1.0f + expf(-z1));
        dout[2 * b] = (sig - lab) / B;
        dout[2 * b + 1] = 2.0f * lab * (z2 - tgt) / cnt;
        l += (fmaxf(z1, 0.0f) - z1 * lab + log1pf(expf(-fabsf(z1)))) / B +
             lab * (z2 - tgt) * (z2 - tgt) / cnt;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0];
}

// dW[o][i] = sum_b dz[b][o] in[b][i]; db[o] = sum_b dz[b][o]  (thread per (o, i), i == I for db)
__global__ void k_linear_bwd_w(const float *dz, const float *in, float *dW, float *db, int B, int I, int O)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= O * (I + 1)) return;
    const int o = idx / (I + 1), i = idx % (I + 1);
    float s = 0.0f;
    if (i < I) {
        for (int b = 0; b < B; ++b) s += dz[(long)b * O + o] * in[(long)b * I + i];
        dW[(long)o * I + i] = s;
    } else {
        for (int b = 0; b < B; ++b) s += dz[(long)b * O + o];
        db[o] = s;
    }
}

// dprev[b][i] = (sum_o dz[b][o] W[o][i]) * GELU'(zprev[b][i])
__global__ void k_linear_bwd_in(const float *dz, const float *W, const float *zprev, float *dprev, int B,
                                int I, int O)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * I) return;
    const int b = idx / I, i = idx % I;
    float s = 0.0f;
    for (int o = 0; o < O; ++o) s += dz[(long)b * O + o] * W[(long)o * I + i];
    dprev[idx] = s * gelu_grad(zprev[idx]);
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
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

unsigned blocks(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct kg_mlp_s {
    int H = 0, maxB = 0;
    size_t np = 0;
    hipStream_t st = nullptr;
    void *mem = nullptr;
    Norm norm{{0, 0, 0, 0}, {1, 1, 1, 1}};
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *xs = nullptr, *z1 = nullptr, *a1 = nullptr, *z2 = nullptr, *a2 = nullptr, *out = nullptr,
          *dout = nullptr, *dz2 = nullptr, *dz1 = nullptr, *loss = nullptr;
    long t = 0;  // Adam steps taken
    std::string err;
    // parameter blocks
    float *W1() { return p; }
    float *b1() { return W1() + (size_t)H * NIN; }
    float *W2() { return b1() + H; }
    float *b2() { return W2() + (size_t)H * H; }
    float *W3() { return b2() + H; }
    float *b3() { return W3() + (size_t)NOUT * H; }
    float *gW1() { return g; }
    float *gb1() { return gW1() + (size_t)H * NIN; }
    float *gW2() { return gb1() + H; }
    float *gb2() { return gW2() + (size_t)H * H; }
    float *gW3() { return gb2() + H; }
    float *gb3() { return gW3() + (size_t)NOUT * H; }
};

namespace {

kg_status mfail(kg_mlp_s *m, kg_status s, const std::string &msg)
{
    if (m) m->err = msg;
    return s;
}

#define MCHK(m, expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return mfail((m), KG_E_HIP, std::string(#expr) + ": " +         \
                                                               hipGetErrorString(e_));        \
    } while (0)

// The three layers for B standardised rows xs: parameters p (flat layout),
// pre-activations z1, z2 and activations a1, a2 (z may alias a when only the
// output is wanted), outputs out.
void layers(hipStream_t st, int H, const float *p, const float *xs, float *z1, float *a1, float *z2,
            float *a2, float *out, int B)
{
    const float *W1 = p, *b1 = W1 + (size_t)H * NIN, *W2 = b1 + H, *b2 = W2 + (size_t)H * H,
                *W3 = b2 + H, *b3 = W3 + (size_t)NOUT * H;
    hipLaunchKernelGGL(k_linear_fwd, dim3(blocks((long)B * H)), dim3(256), 0, st, xs, W1, b1, z1, a1,
                       B, NIN, H, 1);
    hipLaunchKernelGGL(k_linear_fwd, dim3(blocks((long)B * H)), dim3(256), 0, st, a1, W2, b2, z2, a2,
                       B, H, H, 1);
    hipLaunchKernelGGL(k_linear_fwd, dim3(blocks((long)B * NOUT)), dim3(256), 0, st, a2, W3, b3, out,
                       out, B, H, NOUT, 0);
}

// Forward of B <= maxB standardised rows already in m->xs.
void forward(kg_mlp_s *m, int B)
{
    layers(m->st, m->H, m->p, m->xs, m->z1, m->a1, m->z2, m->a2, m->out, B);
}

// Scratch of kg_mlp_forward_noalloc: the standardised inputs and both hidden
// activations of one chunk of rows.  Each GPU holds its own copy; host code
// uses only the per-device addresses from hipGetSymbolAddress.
constexpr size_t NOALLOC_SCRATCH_FLOATS = KG_MLP_NOALLOC_SCRATCH_BYTES / sizeof(float);
static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float *scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per
// device (on that device's first call).
hipError_t scratch_address(float **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = (float *)p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

void backward(kg_mlp_s *m, const float *d_y, int B)
{
    const int H = m->H;
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, m->st, m->out, d_y, m->dout, m->loss, B);
    hipLaunchKernelGGL(k_linear_bwd_w, dim3(blocks((long)NOUT * (H + 1))), dim3(256), 0, m->st, m->dout,
                       m->a2, m->gW3(), m->gb3(), B, H, NOUT);
    hipLaunchKernelGGL(k_linear_bwd_in, dim3(blocks((long)B * H)), dim3(256), 0, m->st, m->dout, m->W3(),
                       m->z2, m->dz2, B, H, NOUT);
    hipLaunchKernelGGL(k_linear_bwd_w, dim3(blocks((long)H * (H + 1))), dim3(256), 0, m->st, m->dz2,
                       m->a1, m->gW2(), m->gb2(), B, H, H);
    hipLaunchKernelGGL(k_linear_bwd_in, dim3(blocks((long)B * H)), dim3(256), 0, m->st, m->dz2, m->W2(),
                       m->z1, m->dz1, B, H, H);
    hipLaunchKernelGGL(k_linear_bwd_w, dim3(blocks((long)H * (NIN + 1))), dim3(256), 0, m->st, m->dz1,
                       m->xs, m->gW1(), m->gb1(), B, NIN, H);
}

}  // namespace

extern "C" {

size_t kg_mlp_num_params(int hidden)
{
    if (hidden < 1) return 0;
    return (size_t)hidden * NIN + hidden + (size_t)hidden * hidden + hidden + (size_t)NOUT * hidden + NOUT;
}

kg_status kg_mlp_create(int hidden, int max_batch, const float *init_params, void *hip_stream,
                        kg_mlp_t **out)
{
    if (!out || !init_params || hidden < 1 || hidden > 1024 || max_batch < 1) return KG_E_INVALID;
    *out = nullptr;
    kg_mlp_s *m = new (std::nothrow) kg_mlp_s();
    if (!m) return KG_E_NOMEM;
    m->H = hidden;
    m->maxB = max_batch;
    m->np = kg_mlp_num_params(hidden);
    m->st = (hipStream_t)hip_stream;
    const size_t B = max_batch, H = hidden;
    const size_t nfl = 4 * m->np + B * NIN + 4 * B * H + 2 * B * NOUT + 2 * B * H + 1;
    if (hipMalloc(&m->mem, nfl * sizeof(float)) != hipSuccess) {
        delete m;
        return KG_E_NOMEM;
    }
    float *c = (float *)m->mem;
    m->p = c; c += m->np;
    m->g = c; c += m->np;
    m->m = c; c += m->np;
    m->v = c; c += m->np;
    m->xs = c; c += B * NIN;
    m->z1 = c; c += B * H;
    m->a1 = c; c += B * H;
    m->z2 = c; c += B * H;
    m->a2 = c; c += B * H;
    m->out = c; c += B * NOUT;
    m->dout = c; c += B * NOUT;
    m->dz2 = c; c += B * H;
    m->dz1 = c; c += B * H;
    m->loss = c;
    std::vector<float> zeros(2 * m->np, 0.0f);
    hipError_t e = hipMemcpyAsync(m->p, init_params, m->np * sizeof(float), hipMemcpyHostToDevice, m->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->m, zeros.data(), 2 * m->np * sizeof(float), hipMemcpyHostToDevice, m->st);
    if (e == hipSuccess) e = hipStreamSynchronize(m->st);
    if (e != hipSuccess) {
        kg_mlp_destroy(m);
        return KG_E_HIP;
    }
    *out = m;
    return KG_OK;
}

void kg_mlp_destroy(kg_mlp_t *m)
{
    if (!m) return;
    if (m->mem) (void)hipFree(m->mem);
    delete m;
}

const char *kg_mlp_last_error(const kg_mlp_t *m) { return m ? m->err.c_str() : "no network"; }

kg_status kg_mlp_set_norm(kg_mlp_t *m, const float *mean, const float *stdev)
{
    if (!m || !mean || !stdev) return KG_E_INVALID;
    for (int i = 0; i < NIN; ++i)
        if (!(stdev[i] > 0)) return mfail(m, KG_E_INVALID, "standard deviations must be > 0");
    for (int i = 0; i < NIN; ++i) {
        m->norm.mean[i] = mean[i];
        m->norm.stdev[i] = stdev[i];
    }
    return KG_OK;
}

kg_status kg_mlp_get_params(kg_mlp_t *m, float *host_out)
{
    if (!m || !host_out) return KG_E_INVALID;
    MCHK(m, hipMemcpyAsync(host_out, m->p, m->np * sizeof(float), hipMemcpyDeviceToHost, m->st));
    MCHK(m, hipStreamSynchronize(m->st));
    return KG_OK;
}

kg_status kg_mlp_forward(kg_mlp_t *m, const float *d_x, int n, float *d_out)
{
    if (!m || !d_x || !d_out || n < 0) return KG_E_INVALID;
    for (int s = 0; s < n; s += m->maxB) {
        const int B = n - s < m->maxB ? n - s : m->maxB;
        hipLaunchKernelGGL(k_standardize, dim3(blocks((long)B * NIN)), dim3(256), 0, m->st,
                           d_x + (long)s * NIN, m->norm, m->xs, B);
        forward(m, B);
        MCHK(m, hipMemcpyAsync(d_out + (long)s * NOUT, m->out, (size_t)B * NOUT * sizeof(float),
                               hipMemcpyDeviceToDevice, m->st));
    }
    MCHK(m, hipGetLastError());
    return KG_OK;
}

kg_status kg_mlp_forward_noalloc(int hidden, const float *d_params, const float *mean,
                                 const float *stdev, const float *d_x, int n, float *d_out,
                                 void *hip_stream)
{
    if (!d_params || n < 0 || (n > 0 && (!d_x || !d_out))) return KG_E_INVALID;
    if (hidden < 1 || hidden > KG_MLP_NOALLOC_MAX_HIDDEN) return KG_E_INVALID;
    Norm norm{{0, 0, 0, 0}, {1, 1, 1, 1}};
    for (int i = 0; i < NIN; ++i) {
        if (mean) norm.mean[i] = mean[i];
        if (stdev) {
            if (!(stdev[i] > 0)) return KG_E_INVALID;
            norm.stdev[i] = stdev[i];
        }
    }
    float *sc = nullptr;
    if (scratch_address(&sc) != hipSuccess) return KG_E_HIP;
    // rows per chunk: standardised inputs and two activation rows each
    const size_t per_row = NIN + 2 * (size_t)hidden;
    const int chunk = (int)(NOALLOC_SCRATCH_FLOATS / per_row);
    hipStream_t st = (hipStream_t)hip_stream;
    float *xs = sc, *a1 = xs + (size_t)chunk * NIN, *a2 = a1 + (size_t)chunk * hidden;
    for (int s = 0; s < n; s += chunk) {
        const int B = n - s < chunk ? n - s : chunk;
        hipLaunchKernelGGL(k_standardize, dim3(blocks((long)B * NIN)), dim3(256), 0, st,
                           d_x + (long)s * NIN, norm, xs, B);
        // pre-activations are not kept: z aliases a; the last layer writes
        // straight into the caller's output
        layers(st, hidden, d_params, xs, a1, a1, a2, a2, d_out + (long)s * NOUT, B);
    }
    return hipGetLastError() == hipSuccess ? KG_OK : KG_E_HIP;
}

kg_status kg_mlp_grad(kg_mlp_t *m, const float *d_x, const float *d_y, int B, float *host_loss,
                      float *host_grads)
{
    if (!m || !d_x || !d_y || B < 1 || B > m->maxB) return KG_E_INVALID;
    hipLaunchKernelGGL(k_standardize, dim3(blocks((long)B * NIN)), dim3(256), 0, m->st, d_x, m->norm,
                       m->xs, B);
    forward(m, B);
    backward(m, d_y, B);
    MCHK(m, hipGetLastError());
    if (host_loss) MCHK(m, hipMemcpyAsync(host_loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->st));
    if (host_grads)
        MCHK(m, hipMemcpyAsync(host_grads, m->g, m->np * sizeof(float), hipMemcpyDeviceToHost, m->st));
    if (host_loss || host_grads) MCHK(m, hipStreamSynchronize(m->st));
    return KG_OK;
}

kg_status kg_mlp_train_step(kg_mlp_t *m, const float *d_x, const float *d_y, int B, float lr,
                            float *host_loss)
{
    kg_status s = kg_mlp_grad(m, d_x, d_y, B, nullptr, nullptr);
    if (s != KG_OK) return s;
    m->t += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)m->t));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)m->t));
    hipLaunchKernelGGL(k_adam, dim3(blocks((long)m->np)), dim3(256), 0, m->st, m->p, m->g, m->m, m->v,
                       (int)m->np, lr, b1, b2, eps, c1, c2);
    MCHK(m, hipGetLastError());
    if (host_loss) {
        MCHK(m, hipMemcpyAsync(host_loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->st));
        MCHK(m, hipStreamSynchronize(m->st));
    }
    return KG_OK;
}

}  // extern "C"
