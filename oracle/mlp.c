/*
 * mlp.c -- FP64 reference of the small multilayer perceptron used as a learned flux correction.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c). Plain loops, float64, no blocking.
 *
 * Network of the learned flux correction (a component the paper does not have):
 *   h1 = silu(W1 x + b1), h2 = silu(W2 h1 + b2), h3 = silu(W3 h2 + b3), y = W4 h3 + b4,
 * with x in R^32, hidden width H, y in R^8 and silu(z) = z / (1 + exp(-z)). Parameters are one flat
 * vector in the order W1[H][32], b1[H], W2[H][H], b2[H], W3[H][H], b3[H], W4[8][H], b4[8] (weights
 * row-major, output index first). Loss: L = 1/(8N) sum_n sum_o (y_no - t_no)^2.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NIN 32
#define NOUT 8

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double silu_grad(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

long mlp_n_params(int H) { return (long)H * NIN + H + 2L * ((long)H * H + H) + (long)NOUT * H + NOUT; }

typedef struct {
    const double *W[4], *b[4];
    int nin[4], nout[4];
} layers;

static layers view(const double *p, int H)
{
    layers L;
    int in[4] = {NIN, H, H, H}, out[4] = {H, H, H, NOUT};
    for (int l = 0; l < 4; l++) {
        L.nin[l] = in[l];
        L.nout[l] = out[l];
        L.W[l] = p;
        p += (long)out[l] * in[l];
        L.b[l] = p;
        p += out[l];
    }
    return L;
}

/* y[N][8] from x[N][32]. */
void mlp_forward(const double *params, int H, int N, const double *x, double *y)
{
    layers L = view(params, H);
    double *prev = malloc(sizeof(double) * (size_t)H), *next = malloc(sizeof(double) * (size_t)H);
    for (int n = 0; n < N; n++) {
        const double *in = x + (size_t)n * NIN;
        for (int l = 0; l < 4; l++) {
            double *out = l < 3 ? next : y + (size_t)n * NOUT;
            for (int o = 0; o < L.nout[l]; o++) {
                double s = L.b[l][o];
                for (int i = 0; i < L.nin[l]; i++) s += L.W[l][(size_t)o * L.nin[l] + i] * in[i];
                out[o] = l < 3 ? silu(s) : s;
            }
            if (l < 3) {
                double *sw = prev;
                prev = next;
                next = sw;
                in = prev;
            }
        }
    }
    free(prev);
    free(next);
}

/* Loss and its gradient with respect to every parameter (grad has mlp_n_params(H) entries). */
double mlp_loss_grad(const double *params, int H, int N, const double *x, const double *t, double *grad)
{
    layers L = view(params, H);
    long np = mlp_n_params(H);
    memset(grad, 0, sizeof(double) * (size_t)np);
    layers G = view(grad, H);
    double *act[4], *pre[4];
    for (int l = 0; l < 4; l++) {
        pre[l] = malloc(sizeof(double) * (size_t)L.nout[l]);
        act[l] = malloc(sizeof(double) * (size_t)L.nout[l]);
    }
    double *dcur = malloc(sizeof(double) * (size_t)H), *dprev = malloc(sizeof(double) * (size_t)H);
    double loss = 0.0;
    const double scale = 1.0 / (8.0 * (double)N);
    for (int n = 0; n < N; n++) {
        const double *xin = x + (size_t)n * NIN;
        /* forward, keeping pre-activations and activations of every layer */
        for (int l = 0; l < 4; l++) {
            const double *in = l == 0 ? xin : act[l - 1];
            for (int o = 0; o < L.nout[l]; o++) {
                double s = L.b[l][o];
                for (int i = 0; i < L.nin[l]; i++) s += L.W[l][(size_t)o * L.nin[l] + i] * in[i];
                pre[l][o] = s;
                act[l][o] = l < 3 ? silu(s) : s;
            }
        }
        /* dL/dy */
        for (int o = 0; o < NOUT; o++) {
            double r = act[3][o] - t[(size_t)n * NOUT + o];
            loss += r * r * scale;
            dcur[o] = 2.0 * r * scale;
        }
        /* backward through the layers */
        for (int l = 3; l >= 0; l--) {
            const double *in = l == 0 ? xin : act[l - 1];
            for (int o = 0; o < L.nout[l]; o++) {
                double g = dcur[o];
                ((double *)G.b[l])[o] += g;
                for (int i = 0; i < L.nin[l]; i++) ((double *)G.W[l])[(size_t)o * L.nin[l] + i] += g * in[i];
            }
            if (l == 0) break;
            for (int i = 0; i < L.nin[l]; i++) {
                double s = 0.0;
                for (int o = 0; o < L.nout[l]; o++) s += L.W[l][(size_t)o * L.nin[l] + i] * dcur[o];
                dprev[i] = s * silu_grad(pre[l - 1][i]);
            }
            double *sw = dcur;
            dcur = dprev;
            dprev = sw;
        }
    }
    for (int l = 0; l < 4; l++) {
        free(pre[l]);
        free(act[l]);
    }
    free(dcur);
    free(dprev);
    return loss;
}

/* One Adam step (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
void mlp_adam(double *p, double *m, double *v, const double *g, long n, double lr, double b1, double b2, double eps,
              int t)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (long i = 0; i < n; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
