/*
 * FP64 reference of the small network used by the learned-weights form.
 *
 * TEST INFRASTRUCTURE ONLY: checks the GPU training and inference kernels.
 *
 * The network is not part of the paper.  It replaces the nonlinear weights
 * of eq. (19) (computed by eq. (28) in the paper) with a prediction:
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3,
 *   left weights = softmax(z[0..3]), right weights = softmax(z[4..7]),
 *   confidence = sigmoid(z[8]).
 * Loss per sample: the squared error of the value each head reconstructs
 * (its weights applied to the candidates of eq. (20) on the normalised
 * stencil) against the value the target weights give, plus binary
 * cross-entropy of the confidence against its label.  The candidates come
 * from or_weno_candidates.  Plain loops, no blocking; the gradient is the
 * chain rule written out.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define NI OR_MLP_NI
#define H OR_MLP_H
#define NO OR_MLP_NO

typedef struct {
  const double *W1, *b1, *W2, *b2, *W3, *b3;
} net_view;

static net_view view(const double *p) {
  net_view v;
  v.W1 = p;
  v.b1 = v.W1 + H * NI;
  v.W2 = v.b1 + H;
  v.b2 = v.W2 + H * H;
  v.W3 = v.b2 + H;
  v.b3 = v.W3 + NO * H;
  return v;
}

static void forward1(const net_view *v, const double *x, double *a1,
                     double *h1, double *a2, double *h2, double *z) {
  int i, k;
  for (i = 0; i < H; i++) {
    double s = v->b1[i];
    for (k = 0; k < NI; k++) s += v->W1[i * NI + k] * x[k];
    a1[i] = s;
    h1[i] = s > 0.0 ? s : 0.0;
  }
  for (i = 0; i < H; i++) {
    double s = v->b2[i];
    for (k = 0; k < H; k++) s += v->W2[i * H + k] * h1[k];
    a2[i] = s;
    h2[i] = s > 0.0 ? s : 0.0;
  }
  for (i = 0; i < NO; i++) {
    double s = v->b3[i];
    for (k = 0; k < H; k++) s += v->W3[i * H + k] * h2[k];
    z[i] = s;
  }
}

void or_mlp_forward(const double *params, const double *X, long n,
                    double *logits) {
  const net_view v = view(params);
  long s;
  for (s = 0; s < n; s++) {
    double a1[H], h1[H], a2[H], h2[H];
    forward1(&v, X + s * NI, a1, h1, a2, h2, logits + s * NO);
  }
}

static void softmax4(const double *z, double *p) {
  double m = z[0], sum = 0.0;
  int k;
  for (k = 1; k < 4; k++)
    if (z[k] > m) m = z[k];
  for (k = 0; k < 4; k++) {
    p[k] = exp(z[k] - m);
    sum += p[k];
  }
  for (k = 0; k < 4; k++) p[k] /= sum;
}

double or_mlp_loss_grad(const double *params, const double *X, const double *Y,
                        const double *C, long n, double *grad) {
  const net_view v = view(params);
  double *gW1 = grad, *gb1 = gW1 + H * NI, *gW2 = gb1 + H, *gb2 = gW2 + H * H,
         *gW3 = gb2 + H, *gb3 = gW3 + NO * H;
  double loss = 0.0;
  long s;
  int i, k;
  memset(grad, 0, sizeof(double) * OR_MLP_NPARAM);
  if (n <= 0) return 0.0;
  for (s = 0; s < n; s++) {
    const double *x = X + s * NI, *y = Y + s * 8;
    double a1[H], h1[H], a2[H], h2[H], z[NO], dz[NO], dh2[H], dh1[H];
    double pl[4], pr[4];
    forward1(&v, x, a1, h1, a2, h2, z);
    softmax4(z, pl);
    softmax4(z + 4, pr);
    {
      /* candidates on the normalised stencil: left from x0..x4, right from
       * the mirror image x5..x1 */
      const double vl[5] = {x[0], x[1], x[2], x[3], x[4]};
      const double vr[5] = {x[5], x[4], x[3], x[2], x[1]};
      double cl[4], cr[4], qhl = 0.0, qhr = 0.0, qtl = 0.0, qtr = 0.0, el, er, c;
      or_weno_candidates(vl, cl);
      or_weno_candidates(vr, cr);
      for (k = 0; k < 4; k++) {
        qhl += pl[k] * cl[k];
        qhr += pr[k] * cr[k];
        qtl += y[k] * cl[k];
        qtr += y[4 + k] * cr[k];
      }
      el = (qhl - qtl) / OR_MLP_VALUE_SCALE;
      er = (qhr - qtr) / OR_MLP_VALUE_SCALE;
      loss += el * el + er * er;
      /* d qhat / d z_k = p_k (c_k - qhat) (softmax Jacobian) */
      for (k = 0; k < 4; k++) {
        dz[k] = 2.0 * el / OR_MLP_VALUE_SCALE * pl[k] * (cl[k] - qhl);
        dz[4 + k] = 2.0 * er / OR_MLP_VALUE_SCALE * pr[k] * (cr[k] - qhr);
      }
      if (C)
        c = C[s];
      else
        c = (fabs(qhl - qtl) < OR_MLP_CONF_TOL && fabs(qhr - qtr) < OR_MLP_CONF_TOL) ? 1.0 : 0.0;
      {
        const double zc = z[8];
        const double sig = 1.0 / (1.0 + exp(-zc));
        /* -[c log sig + (1-c) log(1-sig)], written stably */
        loss += (zc > 0.0 ? zc : 0.0) - zc * c + log1p(exp(-fabs(zc)));
        dz[8] = sig - c;
      }
    }
    for (i = 0; i < NO; i++) dz[i] /= (double)n;
    for (i = 0; i < NO; i++) {
      gb3[i] += dz[i];
      for (k = 0; k < H; k++) gW3[i * H + k] += dz[i] * h2[k];
    }
    for (k = 0; k < H; k++) {
      double t = 0.0;
      for (i = 0; i < NO; i++) t += v.W3[i * H + k] * dz[i];
      dh2[k] = a2[k] > 0.0 ? t : 0.0;
    }
    for (i = 0; i < H; i++) {
      gb2[i] += dh2[i];
      for (k = 0; k < H; k++) gW2[i * H + k] += dh2[i] * h1[k];
    }
    for (k = 0; k < H; k++) {
      double t = 0.0;
      for (i = 0; i < H; i++) t += v.W2[i * H + k] * dh2[i];
      dh1[k] = a1[k] > 0.0 ? t : 0.0;
    }
    for (i = 0; i < H; i++) {
      gb1[i] += dh1[i];
      for (k = 0; k < NI; k++) gW1[i * NI + k] += dh1[i] * x[k];
    }
  }
  return loss / (double)n;
}
