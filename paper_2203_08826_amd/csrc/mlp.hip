// Fully connected network (ReLU hidden layers, linear scalar output) for the
// fusion cost model: forward, mean-squared-error backward and Adam (Kingma
// and Ba, arXiv:1412.6980), FP32 on caller-owned device buffers.
//
// The network is tiny (widths <= 256, batch <= a few thousand), so every
// kernel maps one thread to one output element and sums in a fixed order:
// results are reproducible run to run.
#include "qsv_internal.h"

namespace qsv {

constexpr int MLP_MAX_WIDTH = 256;
constexpr int MLP_T = 256;

// Y[b][o] = act(sum_i X[b][i] W[i][o] + bias[o])
__global__ void k_mlp_layer(const float *__restrict__ X, const float *__restrict__ W, const float *__restrict__ bias,
                            float *__restrict__ Y, int B, int fin, int fout, int relu) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * fout) return;
    const int b = idx / fout, o = idx % fout;
    float s = bias[o];
    for (int i = 0; i < fin; ++i) s = fmaf(X[b * fin + i], W[i * fout + o], s);
    Y[idx] = relu ? fmaxf(s, 0.0f) : s;
}

__global__ void k_mlp_copy(const float *src, float *dst, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = src[i];
}

// dZ = 2 (pred - target) / B
__global__ void k_mlp_out_grad(const float *pred, const float *target, float *dZ, int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) dZ[b] = 2.0f * (pred[b] - target[b]) / (float)B;
}

// dW[i][o] = sum_b A[b][i] dZ[b][o]; db[o] = sum_b dZ[b][o]
__global__ void k_mlp_wgrad(const float *__restrict__ A, const float *__restrict__ dZ, float *__restrict__ dW,
                            float *__restrict__ db, int B, int fin, int fout) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < fin * fout) {
        const int i = idx / fout, o = idx % fout;
        float s = 0.0f;
        for (int b = 0; b < B; ++b) s = fmaf(A[b * fin + i], dZ[b * fout + o], s);
        dW[idx] = s;
    } else if (idx < fin * fout + fout) {
        const int o = idx - fin * fout;
        float s = 0.0f;
        for (int b = 0; b < B; ++b) s += dZ[b * fout + o];
        db[o] = s;
    }
}

// dZprev[b][i] = (sum_o dZ[b][o] W[i][o]) * (A[b][i] > 0)   (A = ReLU output)
__global__ void k_mlp_dact(const float *__restrict__ dZ, const float *__restrict__ W, const float *__restrict__ A,
                           float *__restrict__ dZprev, int B, int fin, int fout) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * fin) return;
    const int b = idx / fin, i = idx % fin;
    float s = 0.0f;
    for (int o = 0; o < fout; ++o) s = fmaf(dZ[b * fout + o], W[i * fout + o], s);
    dZprev[idx] = A[idx] > 0.0f ? s : 0.0f;
}

__global__ void k_mlp_adam(float *p, const float *g, float *m, float *v, int count, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mhat = mi / c1, vhat = vi / c2;
    p[i] -= lr * mhat / (sqrtf(vhat) + eps);
}

static unsigned nb(int count) { return (unsigned)((count + MLP_T - 1) / MLP_T); }

int mlp_check_sizes(const int *sizes, int nlayers) {
    if (!sizes) return fail(QSV_ERR_NULL, "sizes is NULL");
    if (nlayers < 1 || nlayers > 8) return fail(QSV_ERR_ARG, "nlayers must be in [1, 8]");
    for (int l = 0; l <= nlayers; ++l)
        if (sizes[l] < 1 || sizes[l] > MLP_MAX_WIDTH) return fail(QSV_ERR_ARG, "layer widths must be in [1, 256]");
    if (sizes[nlayers] != 1) return fail(QSV_ERR_ARG, "the output width must be 1");
    return QSV_OK;
}

int mlp_param_count(const int *sizes, int nlayers) {
    int c = 0;
    for (int l = 0; l < nlayers; ++l) c += sizes[l] * sizes[l + 1] + sizes[l + 1];
    return c;
}

int mlp_forward(const float *params, const int *sizes, int nlayers, const float *X, int B, float *acts, float *pred,
                hipStream_t s) {
    const float *in = X;
    size_t po = 0, ao = 0;
    for (int l = 0; l < nlayers; ++l) {
        const int fin = sizes[l], fout = sizes[l + 1];
        const float *W = params + po;
        const float *bias = W + (size_t)fin * fout;
        float *Y = acts + ao;
        hipLaunchKernelGGL(k_mlp_layer, dim3(nb(B * fout)), dim3(MLP_T), 0, s, in, W, bias, Y, B, fin, fout,
                           l < nlayers - 1 ? 1 : 0);
        po += (size_t)fin * fout + fout;
        ao += (size_t)B * fout;
        in = Y;
    }
    hipLaunchKernelGGL(k_mlp_copy, dim3(nb(B)), dim3(MLP_T), 0, s, in, pred, B);
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

int qsv_mlp_param_count(const int *sizes, int nlayers) {
    int st = mlp_check_sizes(sizes, nlayers);
    if (st) return st;
    return mlp_param_count(sizes, nlayers);
}

int qsv_mlp_forward(const float *params, const int *sizes, int nlayers, const float *X, int batch, float *acts,
                    float *pred, void *stream) {
    int st = mlp_check_sizes(sizes, nlayers);
    if (st) return st;
    if (!params || !X || !acts || !pred) return fail(QSV_ERR_NULL, "NULL buffer");
    if (batch < 1 || batch > (1 << 20)) return fail(QSV_ERR_ARG, "batch must be in [1, 2^20]");
    return mlp_forward(params, sizes, nlayers, X, batch, acts, pred, (hipStream_t)stream);
}

int qsv_mlp_backward(const float *params, const int *sizes, int nlayers, const float *X, int batch, const float *acts,
                     const float *pred, const float *target, float *grads, float *scratch, void *stream) {
    int st = mlp_check_sizes(sizes, nlayers);
    if (st) return st;
    if (!params || !X || !acts || !pred || !target || !grads || !scratch) return fail(QSV_ERR_NULL, "NULL buffer");
    if (batch < 1 || batch > (1 << 20)) return fail(QSV_ERR_ARG, "batch must be in [1, 2^20]");
    hipStream_t s = (hipStream_t)stream;
    const int B = batch;
    int maxw = 1;
    for (int l = 0; l <= nlayers; ++l) maxw = std::max(maxw, sizes[l]);
    float *dZ = scratch, *dZp = scratch + (size_t)B * maxw;
    // offsets of each layer's params and activations
    std::vector<size_t> po(nlayers), ao(nlayers);
    size_t p = 0, a = 0;
    for (int l = 0; l < nlayers; ++l) {
        po[l] = p;
        ao[l] = a;
        p += (size_t)sizes[l] * sizes[l + 1] + sizes[l + 1];
        a += (size_t)B * sizes[l + 1];
    }
    hipLaunchKernelGGL(k_mlp_out_grad, dim3(nb(B)), dim3(MLP_T), 0, s, pred, target, dZ, B);
    for (int l = nlayers - 1; l >= 0; --l) {
        const int fin = sizes[l], fout = sizes[l + 1];
        const float *Aprev = l == 0 ? X : acts + ao[l - 1];
        float *dW = grads + po[l];
        float *db = dW + (size_t)fin * fout;
        hipLaunchKernelGGL(k_mlp_wgrad, dim3(nb(fin * fout + fout)), dim3(MLP_T), 0, s, Aprev, dZ, dW, db, B, fin,
                           fout);
        if (l > 0) {
            hipLaunchKernelGGL(k_mlp_dact, dim3(nb(B * fin)), dim3(MLP_T), 0, s, dZ, params + po[l], Aprev, dZp, B,
                               fin, fout);
            std::swap(dZ, dZp);
        }
    }
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

int qsv_mlp_adam(float *params, const float *grads, float *m, float *v, int count, int t, float lr, float beta1,
                 float beta2, float eps, void *stream) {
    if (!params || !grads || !m || !v) return fail(QSV_ERR_NULL, "NULL buffer");
    if (count < 1 || t < 1) return fail(QSV_ERR_ARG, "count and t must be >= 1");
    const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_mlp_adam, dim3(nb(count)), dim3(MLP_T), 0, (hipStream_t)stream, params, grads, m, v, count,
                       lr, beta1, beta2, eps, c1, c2);
    QSV_HIP_CHECK(hipGetLastError());
    return QSV_OK;
}

}  // extern "C"
