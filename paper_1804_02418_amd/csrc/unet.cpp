// Host runtime of the warm-start surrogate: the U-Net's layer graph, its
// activation and gradient buffers, and the forward / backward / Adam passes
// built from the kernels of unet_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/rlbm_surrogate.h"
#include "unet_kernels.h"

namespace rlbm {
rlbm_status set_error(rlbm_status st, const char *msg);
}

using namespace rlbm;

namespace {

#define UTRY(expr)                                                                                \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return set_error(RLBM_EDEVICE, (std::string(#expr) + ": " +         \
                                                              hipGetErrorString(e_)).c_str());    \
    } while (0)

inline void ufree(void *p) { (void)hipFree(p); }

struct Layer {
    int ci, co, k, level;
    long long woff, boff;
};

// layer indices in the flat parameter order
enum { E1A, E1B, E2A, E2B, E3A, E3B, E4A, E4B, BA, BB, D4A, D4B, D3A, D3B, D2A, D2B, D1A, D1B, HEAD, NLAYER };

}  // namespace

struct rlbm_unet {
    int base = 0, cin = 0, cout = 0, H = 0, W = 0, maxB = 0;
    hipStream_t stream = nullptr;
    Layer L[NLAYER];
    long long nparam = 0;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    void *theta_bf = nullptr;
    void *wt = nullptr;  // adjoint weights of every 3x3 layer, back to back (adj.toff)
    AdjointTable adj{};
    float *part = nullptr;
    // per-layer regions for the partial sums of the backward pass, reduced
    // in one launch at its end (dpart + wpo[i]: weight-gradient chunks,
    // dpart + bpo[i]: bias rows)
    float *dpart = nullptr;
    long long wpo[NLAYER] = {}, bpo[NLAYER] = {};
    ReduceJobs jobs;
    double *mse_part = nullptr;
    int mse_blocks = 256;
    // activations and their gradients (BF16)
    void *x = nullptr, *gx = nullptr;
    void *act[NLAYER] = {}, *gact[NLAYER] = {};
    void *pool[5] = {}, *gpool[5] = {};  // pool[l]: input of level l (l = 1..4)
    void *cat[4] = {}, *gcat[4] = {};    // cat[l]: input of the decoder block at level l (l = 0..3)
    float *dyb = nullptr;                // head output gradient staging
    int last_batch = 0;
    int adam_t = 0;

    int lh(int l) const { return H >> l; }
    int lw(int l) const { return W >> l; }
};

namespace {

const int kLevel[NLAYER] = {0, 0, 1, 1, 2, 2, 3, 3, 4, 4, 3, 3, 2, 2, 1, 1, 0, 0, 0};

void build_layers(rlbm_unet *N)
{
    const int c0 = N->base, c1 = 2 * c0, c2 = 4 * c0, c3 = 8 * c0;
    const int io[NLAYER][3] = {{N->cin, c0, 3}, {c0, c0, 3}, {c0, c1, 3},      {c1, c1, 3},      {c1, c2, 3},
                               {c2, c2, 3},     {c2, c3, 3}, {c3, c3, 3},      {c3, c3, 3},      {c3, c3, 3},
                               {c3 + c3, c3, 3}, {c3, c3, 3}, {c3 + c2, c2, 3}, {c2, c2, 3},      {c2 + c1, c1, 3},
                               {c1, c1, 3},     {c1 + c0, c0, 3}, {c0, c0, 3},  {c0, N->cout, 1}};
    long long off = 0;
    for (int i = 0; i < NLAYER; ++i) {
        Layer &l = N->L[i];
        l.ci = io[i][0];
        l.co = io[i][1];
        l.k = io[i][2];
        l.level = kLevel[i];
        l.woff = off;
        off += (long long)l.co * l.k * l.k * l.ci;
        l.boff = off;
        off += l.co;
    }
    N->nparam = off;
}

size_t px(const rlbm_unet *N, int level, int B) { return (size_t)B * N->lh(level) * N->lw(level); }

// Seeded He-normal weights (splitmix64 + Box-Muller), zero biases.
void init_params(const rlbm_unet *N, uint64_t seed, std::vector<float> &theta)
{
    theta.assign(N->nparam, 0.f);
    uint64_t s = seed ? seed : 0x9E3779B97F4A7C15ull;
    auto next = [&s]() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto unif = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
    for (int i = 0; i < NLAYER; ++i) {
        const Layer &l = N->L[i];
        const double sd = std::sqrt(2.0 / (l.k * l.k * l.ci));
        for (long long q = 0; q < (long long)l.co * l.k * l.k * l.ci; ++q) {
            const double u1 = unif(), u2 = unif();
            theta[l.woff + q] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    }
}

// Input tensor of a 3x3 layer in the forward graph.
void *layer_input(rlbm_unet *N, int i)
{
    switch (i) {
    case E1A: return N->x;
    case E2A: return N->pool[1];
    case E3A: return N->pool[2];
    case E4A: return N->pool[3];
    case BA: return N->pool[4];
    case D4A: return N->cat[3];
    case D3A: return N->cat[2];
    case D2A: return N->cat[1];
    case D1A: return N->cat[0];
    default: return N->act[i - 1];
    }
}

void *layer_input_grad(rlbm_unet *N, int i)
{
    switch (i) {
    case E1A: return N->gx;
    case E2A: return N->gpool[1];
    case E3A: return N->gpool[2];
    case E4A: return N->gpool[3];
    case BA: return N->gpool[4];
    case D4A: return N->gcat[3];
    case D3A: return N->gcat[2];
    case D2A: return N->gcat[1];
    case D1A: return N->gcat[0];
    default: return N->gact[i - 1];
    }
}

rlbm_status conv_fwd(rlbm_unet *N, int i, int B, const ConvInputs *extra = nullptr)
{
    const Layer &l = N->L[i];
    const char *wbf = static_cast<const char *>(N->theta_bf) + 2 * l.woff;
    ConvInputs x;
    if (extra) x = *extra;
    if (!x.skip) x.in = layer_input(N, i);
    UTRY(conv3x3_forward_ex(x, wbf, N->theta + l.boff, N->act[i], B, N->lh(l.level), N->lw(l.level), l.ci, l.co, true,
                            N->stream));
    return RLBM_OK;
}

// Gradient through layer i's ReLU, its parameters and (when the input
// gradient is wanted) its input.
rlbm_status conv_bwd(rlbm_unet *N, int i, int B, bool want_input)
{
    const Layer &l = N->L[i];
    const int h = N->lh(l.level), w = N->lw(l.level);
    // the partial sums go to the layer's own regions; rlbm_unet_backward
    // reduces every layer's at its end, in one launch
    int rows = 0;
    UTRY(relu_backward_bias_part(N->gact[i], N->act[i], N->dpart + N->bpo[i], N->grad + l.boff,
                                 (long long)B * h * w, l.co, &rows, N->stream));
    if (rows > 0 && !add_reduce_job(N->jobs, N->dpart + N->bpo[i], N->grad + l.boff, l.co, rows))
        return set_error(RLBM_EDEVICE, "rlbm_unet_backward: reduction table full");
    const int chunks = conv3x3_backward_weight_part(N->gact[i], layer_input(N, i), N->dpart + N->wpo[i], B, h, w,
                                                    l.ci, l.co, N->stream);
    if (chunks < 0) return set_error(RLBM_EDEVICE, "rlbm_unet_backward: weight-gradient launch failed");
    if (!add_reduce_job(N->jobs, N->dpart + N->wpo[i], N->grad + l.woff, (long long)l.co * 9 * l.ci, chunks))
        return set_error(RLBM_EDEVICE, "rlbm_unet_backward: reduction table full");
    if (want_input) {
        // the adjoint weights of every layer were formed at the start of the
        // backward pass; layer i is entry i (every layer before the head is 3 x 3)
        const void *wt = static_cast<const char *>(N->wt) + 2 * N->adj.toff[i];
        UTRY(conv3x3_forward(N->gact[i], wt, nullptr, layer_input_grad(N, i), B, h, w, l.co, l.ci, false,
                             N->stream));
    }
    return RLBM_OK;
}

}  // namespace

namespace {
// The kernels read and write BF16 tensors 16 bytes (8 channels) at a time.
bool misaligned16(const void *a, const void *b, const void *c)
{
    return ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c)) & 15) != 0;
}

}  // namespace

extern "C" {

void rlbm_unet_destroy(rlbm_unet *N)
{
    if (!N) return;
    if (N->stream) (void)hipStreamSynchronize(N->stream);
    ufree(N->theta);
    ufree(N->grad);
    ufree(N->m);
    ufree(N->v);
    ufree(N->theta_bf);
    ufree(N->wt);
    ufree(N->part);
    ufree(N->dpart);
    ufree(N->mse_part);
    ufree(N->x);
    ufree(N->gx);
    ufree(N->dyb);
    for (int i = 0; i < NLAYER; ++i) {
        ufree(N->act[i]);
        ufree(N->gact[i]);
    }
    for (int l = 0; l < 5; ++l) {
        ufree(N->pool[l]);
        ufree(N->gpool[l]);
    }
    for (int l = 0; l < 4; ++l) {
        ufree(N->cat[l]);
        ufree(N->gcat[l]);
    }
    delete N;
}

rlbm_status rlbm_unet_create(int base, int cin, int cout, int height, int width, int max_batch, uint64_t seed,
                             void *hip_stream, rlbm_unet **out)
{
    if (!out) return set_error(RLBM_EINVAL, "rlbm_unet_create: out is NULL");
    *out = nullptr;
    if (base < 16 || base % 16 || cin < 16 || cin % 16 || cout < 1 || height < 16 || height % 16 || width < 16 ||
        width % 16 || max_batch < 1)
        return set_error(RLBM_EINVAL, "rlbm_unet_create: base and cin must be multiples of 16, H and W multiples of 16");
    rlbm_unet *N = new (std::nothrow) rlbm_unet();
    if (!N) return set_error(RLBM_ENOMEM, "rlbm_unet_create: host allocation failed");
    N->base = base;
    N->cin = cin;
    N->cout = cout;
    N->H = height;
    N->W = width;
    N->maxB = max_batch;
    N->stream = static_cast<hipStream_t>(hip_stream);
    build_layers(N);
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    const long long P = N->nparam;
    alloc((void **)&N->theta, P * 4);
    alloc((void **)&N->grad, P * 4);
    alloc((void **)&N->m, P * 4);
    alloc((void **)&N->v, P * 4);
    alloc(&N->theta_bf, P * 2);
    size_t part_max = 0;
    // the 3x3 layers' adjoint weights, back to back in layer order
    N->adj.n = 0;
    N->adj.toff[0] = 0;
    for (int i = 0; i < NLAYER; ++i) {
        const Layer &l = N->L[i];
        if (l.k != 3) continue;
        N->adj.woff[N->adj.n] = l.woff;
        N->adj.ci[N->adj.n] = l.ci;
        N->adj.co[N->adj.n] = l.co;
        N->adj.toff[N->adj.n + 1] = N->adj.toff[N->adj.n] + (long long)l.co * 9 * l.ci;
        ++N->adj.n;
    }
    long long dpart_len = 0;
    for (int i = 0; i < NLAYER; ++i) {
        const Layer &l = N->L[i];
        const long long np = (long long)px(N, l.level, max_batch);
        if (l.k == 3) {
            part_max = std::max(part_max, (size_t)conv3x3_wgrad_chunks(max_batch, N->lh(l.level), N->lw(l.level), l.ci, l.co) *
                                              l.co * 9 * l.ci);
            // the layer's regions hold its partials at any batch up to max_batch
            int chunks = 1;
            for (int b = 1; b <= max_batch; ++b)
                chunks = std::max(chunks, conv3x3_wgrad_chunks(b, N->lh(l.level), N->lw(l.level), l.ci, l.co));
            N->wpo[i] = dpart_len;
            dpart_len += (long long)chunks * l.co * 9 * l.ci;
            N->bpo[i] = dpart_len;
            dpart_len += (long long)channel_sum_blocks(np) * l.co;
        }
        // bias sums (and the head's parameter sums): one row per block
        part_max = std::max(part_max, (size_t)channel_sum_blocks(np) * l.co * (l.k == 3 ? 1 : l.ci + 1));
        alloc(&N->act[i], px(N, l.level, max_batch) * l.co * 2);
        alloc(&N->gact[i], px(N, l.level, max_batch) * l.co * 2);
    }
    alloc(&N->wt, (size_t)N->adj.toff[N->adj.n] * 2);
    alloc((void **)&N->part, part_max * 4);
    alloc((void **)&N->dpart, (size_t)dpart_len * 4);
    alloc((void **)&N->mse_part, N->mse_blocks * 8);
    alloc(&N->x, px(N, 0, max_batch) * cin * 2);
    alloc(&N->gx, px(N, 0, max_batch) * cin * 2);
    alloc((void **)&N->dyb, px(N, 0, max_batch) * cout * 4);
    const int c0 = base, c1 = 2 * base, c2 = 4 * base, c3 = 8 * base;
    const int pool_c[5] = {0, c0, c1, c2, c3};
    for (int l = 1; l <= 4; ++l) {
        alloc(&N->pool[l], px(N, l, max_batch) * pool_c[l] * 2);
        alloc(&N->gpool[l], px(N, l, max_batch) * pool_c[l] * 2);
    }
    const int cat_c[4] = {c1 + c0, c2 + c1, c3 + c2, c3 + c3};
    for (int l = 0; l < 4; ++l) {
        alloc(&N->cat[l], px(N, l, max_batch) * cat_c[l] * 2);
        alloc(&N->gcat[l], px(N, l, max_batch) * cat_c[l] * 2);
    }
    if (e != hipSuccess) {
        rlbm_unet_destroy(N);
        return set_error(e == hipErrorOutOfMemory ? RLBM_ENOMEM : RLBM_EDEVICE, hipGetErrorString(e));
    }
    std::vector<float> theta;
    init_params(N, seed, theta);
    rlbm_status st = rlbm_unet_set_params(N, theta.data());
    if (st) {
        rlbm_unet_destroy(N);
        return st;
    }
    *out = N;
    return RLBM_OK;
}

rlbm_status rlbm_unet_param_count(rlbm_unet *N, int64_t *n)
{
    if (!N || !n) return set_error(RLBM_EINVAL, "rlbm_unet_param_count: bad argument");
    *n = N->nparam;
    return RLBM_OK;
}

rlbm_status rlbm_unet_set_params(rlbm_unet *N, const float *theta)
{
    if (!N || !theta) return set_error(RLBM_EINVAL, "rlbm_unet_set_params: bad argument");
    UTRY(hipMemcpyAsync(N->theta, theta, N->nparam * 4, hipMemcpyHostToDevice, N->stream));
    UTRY(to_bf16(N->theta, N->theta_bf, N->nparam, N->stream));
    UTRY(hipMemsetAsync(N->grad, 0, N->nparam * 4, N->stream));
    UTRY(hipMemsetAsync(N->m, 0, N->nparam * 4, N->stream));
    UTRY(hipMemsetAsync(N->v, 0, N->nparam * 4, N->stream));
    UTRY(hipStreamSynchronize(N->stream));
    N->adam_t = 0;
    return RLBM_OK;
}

rlbm_status rlbm_unet_get_params(rlbm_unet *N, float *theta)
{
    if (!N || !theta) return set_error(RLBM_EINVAL, "rlbm_unet_get_params: bad argument");
    UTRY(hipMemcpyAsync(theta, N->theta, N->nparam * 4, hipMemcpyDeviceToHost, N->stream));
    UTRY(hipStreamSynchronize(N->stream));
    return RLBM_OK;
}

rlbm_status rlbm_unet_get_grads(rlbm_unet *N, float *g)
{
    if (!N || !g) return set_error(RLBM_EINVAL, "rlbm_unet_get_grads: bad argument");
    UTRY(hipMemcpyAsync(g, N->grad, N->nparam * 4, hipMemcpyDeviceToHost, N->stream));
    UTRY(hipStreamSynchronize(N->stream));
    return RLBM_OK;
}

rlbm_status rlbm_unet_zero_grad(rlbm_unet *N)
{
    if (!N) return set_error(RLBM_EINVAL, "rlbm_unet_zero_grad: NULL");
    UTRY(hipMemsetAsync(N->grad, 0, N->nparam * 4, N->stream));
    return RLBM_OK;
}

rlbm_status rlbm_unet_forward(rlbm_unet *N, const float *x, float *y, int batch)
{
    if (!N || !x || !y || batch < 1 || batch > N->maxB) return set_error(RLBM_EINVAL, "rlbm_unet_forward: bad argument");
    const int B = batch;
    const int c0 = N->base, c1 = 2 * c0, c2 = 4 * c0, c3 = 8 * c0;
    UTRY(to_bf16(x, N->x, (long long)px(N, 0, B) * N->cin, N->stream));
    rlbm_status st;
    auto block = [&](int a, int b) {
        rlbm_status s2 = conv_fwd(N, a, B);
        return s2 ? s2 : conv_fwd(N, b, B);
    };
    // The pooled inputs of levels 1..4 come out of the last convolution of
    // the level above, the decoder's concatenations are read in place by its
    // first convolution, and the head rides on the last one.
    auto enc = [&](int a, int b, int level) {
        rlbm_status s2 = conv_fwd(N, a, B);
        if (s2) return s2;
        ConvInputs io;
        io.pooled = N->pool[level + 1];
        return conv_fwd(N, b, B, &io);
    };
    auto dec = [&](int a, int b, int up, int skip, int cu) {
        ConvInputs io;
        io.in = N->act[up];
        io.skip = N->act[skip];
        io.cu = cu;
        rlbm_status s2 = conv_fwd(N, a, B, &io);
        return s2 ? s2 : conv_fwd(N, b, B);
    };
    if ((st = enc(E1A, E1B, 0))) return st;
    if ((st = enc(E2A, E2B, 1))) return st;
    if ((st = enc(E3A, E3B, 2))) return st;
    if ((st = enc(E4A, E4B, 3))) return st;
    if ((st = block(BA, BB))) return st;
    if ((st = dec(D4A, D4B, BB, E4B, c3))) return st;
    if ((st = dec(D3A, D3B, D4B, E3B, c3))) return st;
    if ((st = dec(D2A, D2B, D3B, E2B, c2))) return st;
    const Layer &h = N->L[HEAD];
    {
        ConvInputs io;
        io.in = N->act[D2B];
        io.skip = N->act[E1B];
        io.cu = c1;
        if ((st = conv_fwd(N, D1A, B, &io))) return st;
        ConvInputs hx;
        hx.head_w = static_cast<const char *>(N->theta_bf) + 2 * h.woff;
        hx.head_b = N->theta + h.boff;
        hx.head_out = y;
        hx.head_o = h.co;
        if ((st = conv_fwd(N, D1B, B, &hx))) return st;
    }
    N->last_batch = B;
    return RLBM_OK;
}

rlbm_status rlbm_unet_mse(rlbm_unet *N, const float *y, const float *t, int batch, float *loss, float *dy)
{
    if (!N || !y || !t || batch < 1 || batch > N->maxB) return set_error(RLBM_EINVAL, "rlbm_unet_mse: bad argument");
    const long long n = (long long)px(N, 0, batch) * N->cout;
    UTRY(mse(y, t, dy, N->mse_part, N->mse_blocks, n, N->stream));
    std::vector<double> h(N->mse_blocks);
    UTRY(hipMemcpyAsync(h.data(), N->mse_part, h.size() * 8, hipMemcpyDeviceToHost, N->stream));
    UTRY(hipStreamSynchronize(N->stream));
    double s = 0;
    for (double v : h) s += v;
    if (loss) *loss = (float)(s / n);
    return RLBM_OK;
}

rlbm_status rlbm_unet_backward(rlbm_unet *N, const float *dy, int batch, float *dx)
{
    if (!N || !dy || batch != N->last_batch) return set_error(RLBM_EINVAL, "rlbm_unet_backward: needs the last forward's batch");
    const int B = batch;
    const int c0 = N->base, c1 = 2 * c0, c2 = 4 * c0, c3 = 8 * c0;
    const Layer &h = N->L[HEAD];
    UTRY(conv3x3_adjoint_weights_all(N->theta_bf, N->wt, N->adj, N->stream));
    N->jobs = ReduceJobs();
    // the forward read the decoder's concatenations in place; the weight
    // gradients of the decoder's first convolutions want them formed
    UTRY(up_concat(N->act[BB], N->act[E4B], N->cat[3], B, N->lh(3), N->lw(3), c3, c3, N->stream));
    UTRY(up_concat(N->act[D4B], N->act[E3B], N->cat[2], B, N->lh(2), N->lw(2), c3, c2, N->stream));
    UTRY(up_concat(N->act[D3B], N->act[E2B], N->cat[1], B, N->lh(1), N->lw(1), c2, c1, N->stream));
    UTRY(up_concat(N->act[D2B], N->act[E1B], N->cat[0], B, N->lh(0), N->lw(0), c1, c0, N->stream));
    UTRY(head_backward(dy, N->act[D1B], static_cast<const char *>(N->theta_bf) + 2 * h.woff, N->gact[D1B], N->part,
                       N->grad + h.woff, N->grad + h.boff, (long long)px(N, 0, B), h.ci, h.co, N->stream));
    rlbm_status st;
    auto block = [&](int a, int b, bool input) {
        rlbm_status s2 = conv_bwd(N, b, B, true);
        return s2 ? s2 : conv_bwd(N, a, B, input);
    };
    if ((st = block(D1A, D1B, true))) return st;
    UTRY(up_backward(N->gcat[0], N->gact[D2B], B, N->lh(0), N->lw(0), c1, c1 + c0, N->stream));
    if ((st = block(D2A, D2B, true))) return st;
    UTRY(up_backward(N->gcat[1], N->gact[D3B], B, N->lh(1), N->lw(1), c2, c2 + c1, N->stream));
    if ((st = block(D3A, D3B, true))) return st;
    UTRY(up_backward(N->gcat[2], N->gact[D4B], B, N->lh(2), N->lw(2), c3, c3 + c2, N->stream));
    if ((st = block(D4A, D4B, true))) return st;
    UTRY(up_backward(N->gcat[3], N->gact[BB], B, N->lh(3), N->lw(3), c3, c3 + c3, N->stream));
    if ((st = block(BA, BB, true))) return st;
    UTRY(pool_backward(N->gpool[4], N->gcat[3], c3 + c3, c3, N->gact[E4B], B, N->lh(3), N->lw(3), c3, N->stream));
    if ((st = block(E4A, E4B, true))) return st;
    UTRY(pool_backward(N->gpool[3], N->gcat[2], c3 + c2, c3, N->gact[E3B], B, N->lh(2), N->lw(2), c2, N->stream));
    if ((st = block(E3A, E3B, true))) return st;
    UTRY(pool_backward(N->gpool[2], N->gcat[1], c2 + c1, c2, N->gact[E2B], B, N->lh(1), N->lw(1), c1, N->stream));
    if ((st = block(E2A, E2B, true))) return st;
    UTRY(pool_backward(N->gpool[1], N->gcat[0], c1 + c0, c1, N->gact[E1B], B, N->lh(0), N->lw(0), c0, N->stream));
    if ((st = block(E1A, E1B, dx != nullptr))) return st;
    UTRY(reduce_partials(N->jobs, N->stream));
    if (dx) UTRY(to_f32(N->gx, dx, (long long)px(N, 0, B) * N->cin, N->stream));
    return RLBM_OK;
}

rlbm_status rlbm_unet_adam_step(rlbm_unet *N, float lr, float b1, float b2, float eps)
{
    if (!N || !(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return set_error(RLBM_EINVAL, "rlbm_unet_adam_step: bad argument");
    N->adam_t += 1;
    const float c1 = 1.f - std::pow(b1, (float)N->adam_t), c2 = 1.f - std::pow(b2, (float)N->adam_t);
    UTRY(adam(N->theta, N->grad, N->m, N->v, N->theta_bf, N->nparam, lr, b1, b2, eps, c1, c2, N->stream));
    return RLBM_OK;
}

rlbm_status rlbm_conv3x3_forward(const void *x, const void *w, const float *b, void *y, int B, int H, int W, int ci,
                                 int co, int relu, void *stream)
{
    if (!x || !w || !y || ci % 16 || co % 16 || B < 1 || H < 1 || W < 1 || misaligned16(x, w, y))
        return set_error(RLBM_EINVAL, "rlbm_conv3x3_forward: bad argument");
    UTRY(conv3x3_forward(x, w, b, y, B, H, W, ci, co, relu != 0, static_cast<hipStream_t>(stream)));
    return RLBM_OK;
}

rlbm_status rlbm_conv3x3_backward_data(const void *dy, const void *w, void *dx, int B, int H, int W, int ci, int co,
                                       void *stream)
{
    if (!dy || !w || !dx || ci % 16 || co % 16 || B < 1 || H < 1 || W < 1 || misaligned16(dy, w, dx))
        return set_error(RLBM_EINVAL, "rlbm_conv3x3_backward_data: bad argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *wt = nullptr;
    UTRY(hipMalloc(&wt, (size_t)co * 9 * ci * 2));
    hipError_t e = conv3x3_adjoint_weights(w, wt, ci, co, s);
    if (e == hipSuccess) e = conv3x3_forward(dy, wt, nullptr, dx, B, H, W, co, ci, false, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ufree(wt);
    if (e != hipSuccess) return set_error(RLBM_EDEVICE, hipGetErrorString(e));
    return RLBM_OK;
}

rlbm_status rlbm_conv3x3_backward_weight(const void *dy, const void *x, float *gw, float *gb, int B, int H, int W,
                                         int ci, int co, void *stream)
{
    if (!dy || !x || !gw || ci % 16 || co % 16 || B < 1 || H < 1 || W < 1 || misaligned16(dy, x, x))
        return set_error(RLBM_EINVAL, "rlbm_conv3x3_backward_weight: bad argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long np = (long long)B * H * W;
    float *part = nullptr;
    const size_t nw = (size_t)conv3x3_wgrad_chunks(B, H, W, ci, co) * co * 9 * ci, nbias = (size_t)channel_sum_blocks(np) * co;
    UTRY(hipMalloc((void **)&part, std::max(nw, nbias) * 4));
    hipError_t e = conv3x3_backward_weight(dy, x, part, gw, B, H, W, ci, co, s);
    if (e == hipSuccess && gb) e = channel_sum(dy, part, gb, np, co, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ufree(part);
    if (e != hipSuccess) return set_error(RLBM_EDEVICE, hipGetErrorString(e));
    return RLBM_OK;
}

}  // extern "C"
