/*
 * vpmc_mlp.c -- FP64 reference of the learned aperture surrogate's network
 * (forward pass, loss and gradients).  TEST INFRASTRUCTURE ONLY, like the
 * transport oracle: the BF16 MFMA kernels of the product library are
 * checked against it and it shares no code with them.
 *
 * Network: 8 inputs -> 4 hidden layers of 256 SiLU units -> 29 outputs.
 * Outputs: [0] transmission logit; [1..4] mixture-weight logits of 4
 * components; [5..16] component means (3 per component); [17..28] component
 * log standard deviations (3 per component) over the normalised outgoing
 * (energy loss, deflection angle, lateral offset) of a VP that crosses the
 * brass block.
 * Loss per sample: binary cross-entropy of the transmission logit against
 * the observed outcome, plus, for transmitted samples, the negative log
 * likelihood of the outgoing triple under the diagonal Gaussian mixture.
 * Parameters are stored layer by layer as W[out][in] then b[out].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NL 5
static const int DIMS[NL + 1] = {8, 256, 256, 256, 256, 29};
#define NMIX 4
#define NY 3
#define LOG_2PI 1.8378770664093453

int mlp_num_params(void)
{
    int n = 0;
    for (int l = 0; l < NL; l++) n += DIMS[l + 1] * DIMS[l] + DIMS[l + 1];
    return n;
}

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double dsilu(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

/* pre-activations z[l] and activations a[l] of one sample (a[0] = input) */
typedef struct {
    double z[NL][256];
    double a[NL + 1][256];
} trace_t;

static void forward_one(const double *p, const double *x, trace_t *t)
{
    memcpy(t->a[0], x, sizeof(double) * DIMS[0]);
    const double *w = p;
    for (int l = 0; l < NL; l++) {
        int ni = DIMS[l], no = DIMS[l + 1];
        const double *b = w + no * ni;
        for (int o = 0; o < no; o++) {
            double s = b[o];
            for (int i = 0; i < ni; i++) s += w[o * ni + i] * t->a[l][i];
            t->z[l][o] = s;
            t->a[l + 1][o] = (l < NL - 1) ? silu(s) : s;
        }
        w = b + no;
    }
}

void mlp_forward(const double *params, const double *x, int n, double *out)
{
    trace_t *t = malloc(sizeof *t);
    for (int s = 0; s < n; s++) {
        forward_one(params, x + s * DIMS[0], t);
        memcpy(out + s * DIMS[NL], t->a[NL], sizeof(double) * DIMS[NL]);
    }
    free(t);
}

/* loss of one sample and its gradient with respect to the 29 outputs */
static double head_loss(const double *o, const double *y, double trans, double *g)
{
    memset(g, 0, sizeof(double) * DIMS[NL]);
    /* transmission: BCE with logits */
    double lt = o[0];
    double loss = fmax(lt, 0.0) - lt * trans + log1p(exp(-fabs(lt)));
    g[0] = 1.0 / (1.0 + exp(-lt)) - trans;
    if (trans > 0.5) {
        /* mixture NLL: -log sum_c pi_c prod_j N(y_j; mu_cj, sigma_cj) */
        double lw[NMIX], lp[NMIX], m = -INFINITY, mw = -INFINITY;
        for (int c = 0; c < NMIX; c++) mw = fmax(mw, o[1 + c]);
        double zs = 0.0;
        for (int c = 0; c < NMIX; c++) zs += exp(o[1 + c] - mw);
        for (int c = 0; c < NMIX; c++) {
            lw[c] = o[1 + c] - mw - log(zs);                 /* log softmax */
            double s = 0.0;
            for (int j = 0; j < NY; j++) {
                double mu = o[5 + NY * c + j], ls = o[17 + NY * c + j];
                double r = (y[j] - mu) * exp(-ls);
                s += -0.5 * r * r - ls - 0.5 * LOG_2PI;
            }
            lp[c] = lw[c] + s;
            m = fmax(m, lp[c]);
        }
        double tot = 0.0;
        for (int c = 0; c < NMIX; c++) tot += exp(lp[c] - m);
        double lse = m + log(tot);
        loss += -lse;
        for (int c = 0; c < NMIX; c++) {
            double gam = exp(lp[c] - lse);                   /* responsibility */
            double pic = exp(lw[c]);
            g[1 + c] += pic - gam;                           /* d(-lse)/d logit */
            for (int j = 0; j < NY; j++) {
                double mu = o[5 + NY * c + j], ls = o[17 + NY * c + j];
                double iv = exp(-2.0 * ls), d = y[j] - mu;
                g[5 + NY * c + j] += -gam * d * iv;
                g[17 + NY * c + j] += -gam * (d * d * iv - 1.0);
            }
        }
    }
    return loss;
}

/* mean loss over n samples; grad (num_params) receives its gradient */
double mlp_loss_grad(const double *params, const double *x, const double *y, const double *trans, int n,
                     double *grad)
{
    int np = mlp_num_params();
    memset(grad, 0, sizeof(double) * np);
    trace_t *t = malloc(sizeof *t);
    double delta[256], prev[256], go[32];
    double total = 0.0;
    for (int s = 0; s < n; s++) {
        forward_one(params, x + s * DIMS[0], t);
        total += head_loss(t->a[NL], y + s * NY, trans[s], go);
        /* backward: delta = dL/dz of the current layer */
        for (int o = 0; o < DIMS[NL]; o++) delta[o] = go[o] / n;
        /* walk layers from the top: find each layer's parameter offset */
        for (int l = NL - 1; l >= 0; l--) {
            int ni = DIMS[l], no = DIMS[l + 1];
            int off = 0;
            for (int q = 0; q < l; q++) off += DIMS[q + 1] * DIMS[q] + DIMS[q + 1];
            const double *w = params + off;
            double *gw = grad + off, *gb = gw + no * ni;
            for (int o = 0; o < no; o++) {
                gb[o] += delta[o];
                for (int i = 0; i < ni; i++) gw[o * ni + i] += delta[o] * t->a[l][i];
            }
            if (l > 0) {
                for (int i = 0; i < ni; i++) {
                    double s2 = 0.0;
                    for (int o = 0; o < no; o++) s2 += w[o * ni + i] * delta[o];
                    prev[i] = s2 * dsilu(t->z[l - 1][i]);
                }
                memcpy(delta, prev, sizeof(double) * ni);
            }
        }
    }
    free(t);
    return total / n;
}

/* one Adam step (Kingma & Ba): m, v moment estimates, step count t >= 1 */
void mlp_adam_step(double *params, const double *grad, double *m, double *v, int np, int t, double lr,
                   double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int i = 0; i < np; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        params[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
