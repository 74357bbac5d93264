/*
 * mlp_oracle.c -- plain FP64 reference of the per-column closure network.
 *
 * TEST INFRASTRUCTURE ONLY, like ocean_oracle.c: the tests and the smoke check
 * use it to check the GPU's network kernels; the product never links it.
 *
 * The paper motivates learned parameterizations of unresolved processes
 * (Sec. 3: irreducible uncertainties addressed through data and machine
 * learning) and uses a vertical-mixing closure in its runs (Sec. 6). The
 * network here maps a column's features to the vertical diffusivity profile:
 * Linear -> ReLU -> Linear -> ReLU -> Linear, trained on the mean-squared
 * error with Adam. Matrices are row-major: X is n x d_in, W1 is d_in x h1,
 * W2 is h1 x h2, W3 is h2 x d_out; Y = relu(relu(X W1 + b1) W2 + b2) W3 + b3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* C (n x m) = A (n x k) B (k x m) + bias (m), optional ReLU */
static void dense(const double* A, const double* B, const double* bias, int n, int k, int m, int relu, double* C) {
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < m; ++c) {
            double s = bias ? bias[c] : 0.0;
            for (int q = 0; q < k; ++q) s += A[(size_t)r * k + q] * B[(size_t)q * m + c];
            C[(size_t)r * m + c] = (relu && s < 0.0) ? 0.0 : s;
        }
}

/* Forward pass; H1 (n x h1) and H2 (n x h2) keep the post-ReLU activations. */
void orc_mlp_forward(const double* X, int n, int din, int h1, int h2, int dout, const double* W1, const double* b1,
                     const double* W2, const double* b2, const double* W3, const double* b3, double* H1, double* H2,
                     double* Y) {
    dense(X, W1, b1, n, din, h1, 1, H1);
    dense(H1, W2, b2, n, h1, h2, 1, H2);
    dense(H2, W3, b3, n, h2, dout, 0, Y);
}

/* Loss L = sum over the n x d_out entries of (Y - T)^2 / (2 n d_out) and its
 * gradients with respect to every weight and bias (backpropagation through the
 * ReLUs, whose derivative is taken as 0 at 0). Returns L. */
double orc_mlp_backward(const double* X, const double* T, int n, int din, int h1, int h2, int dout, const double* W1,
                        const double* b1, const double* W2, const double* b2, const double* W3, const double* b3,
                        double* gW1, double* gb1, double* gW2, double* gb2, double* gW3, double* gb3) {
    double* H1 = (double*)malloc(sizeof(double) * (size_t)n * h1);
    double* H2 = (double*)malloc(sizeof(double) * (size_t)n * h2);
    double* Y = (double*)malloc(sizeof(double) * (size_t)n * dout);
    double* dY = (double*)malloc(sizeof(double) * (size_t)n * dout);
    double* dH2 = (double*)malloc(sizeof(double) * (size_t)n * h2);
    double* dH1 = (double*)malloc(sizeof(double) * (size_t)n * h1);
    orc_mlp_forward(X, n, din, h1, h2, dout, W1, b1, W2, b2, W3, b3, H1, H2, Y);
    const double scale = 1.0 / ((double)n * dout);
    double loss = 0.0;
    for (size_t e = 0; e < (size_t)n * dout; ++e) {
        double r = Y[e] - T[e];
        loss += 0.5 * r * r * scale;
        dY[e] = r * scale;
    }
    /* layer 3 */
    for (int a = 0; a < h2; ++a)
        for (int c = 0; c < dout; ++c) {
            double s = 0.0;
            for (int r = 0; r < n; ++r) s += H2[(size_t)r * h2 + a] * dY[(size_t)r * dout + c];
            gW3[(size_t)a * dout + c] = s;
        }
    for (int c = 0; c < dout; ++c) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += dY[(size_t)r * dout + c];
        gb3[c] = s;
    }
    for (int r = 0; r < n; ++r)
        for (int a = 0; a < h2; ++a) {
            double s = 0.0;
            for (int c = 0; c < dout; ++c) s += dY[(size_t)r * dout + c] * W3[(size_t)a * dout + c];
            dH2[(size_t)r * h2 + a] = H2[(size_t)r * h2 + a] > 0.0 ? s : 0.0;
        }
    /* layer 2 */
    for (int a = 0; a < h1; ++a)
        for (int c = 0; c < h2; ++c) {
            double s = 0.0;
            for (int r = 0; r < n; ++r) s += H1[(size_t)r * h1 + a] * dH2[(size_t)r * h2 + c];
            gW2[(size_t)a * h2 + c] = s;
        }
    for (int c = 0; c < h2; ++c) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += dH2[(size_t)r * h2 + c];
        gb2[c] = s;
    }
    for (int r = 0; r < n; ++r)
        for (int a = 0; a < h1; ++a) {
            double s = 0.0;
            for (int c = 0; c < h2; ++c) s += dH2[(size_t)r * h2 + c] * W2[(size_t)a * h2 + c];
            dH1[(size_t)r * h1 + a] = H1[(size_t)r * h1 + a] > 0.0 ? s : 0.0;
        }
    /* layer 1 */
    for (int a = 0; a < din; ++a)
        for (int c = 0; c < h1; ++c) {
            double s = 0.0;
            for (int r = 0; r < n; ++r) s += X[(size_t)r * din + a] * dH1[(size_t)r * h1 + c];
            gW1[(size_t)a * h1 + c] = s;
        }
    for (int c = 0; c < h1; ++c) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += dH1[(size_t)r * h1 + c];
        gb1[c] = s;
    }
    free(H1); free(H2); free(Y); free(dY); free(dH2); free(dH1);
    return loss;
}

/* One Adam update (Kingma and Ba 2015) of n parameters at step t >= 1:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
void orc_adam(double* p, const double* g, double* m, double* v, int64_t n, int t, double lr, double beta1,
              double beta2, double eps) {
    const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t q = 0; q < n; ++q) {
        m[q] = beta1 * m[q] + (1.0 - beta1) * g[q];
        v[q] = beta2 * v[q] + (1.0 - beta2) * g[q] * g[q];
        p[q] -= lr * (m[q] / c1) / (sqrt(v[q] / c2) + eps);
    }
}
