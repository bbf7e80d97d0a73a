/*
 * fem_oracle.c -- plain, slow, FP64 CPU reference of the Free-Energy Machine
 * (FEM) step, written from the paper (Shen et al., "Free-Energy Machine for
 * Combinatorial Optimization", arXiv 2412.09285).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or table with the HIP
 * library: it works directly from undirected edge lists and clause lists,
 * never from the library's CSR / incidence structures.
 *
 * Everything is double precision and single-threaded.  Loops follow the
 * definitions in the paper's order; no blocking, fusion or reordering.
 *
 * Readings of the paper taken here:
 *  - Edge sums run over ordered pairs: each undirected edge {i,j} appears as
 *    (i,j) and (j,i).  This is the convention under which the explicit
 *    gradients printed in the supplementary section "The explicit gradients
 *    and manipulated gradients" are derivatives of F, and under which the
 *    stationary points reproduce the mean-field equation m = tanh(beta J m).
 *  - MaxCut and Max-k-SAT use one logit per variable, P_i = sigmoid(h_i)
 *    (supplementary section "Simplification of FEM for solving the MaxCut
 *    problem"); balanced min-cut uses q logits and a softmax (Results,
 *    "Free-Energy Machine").
 *  - The balance term of bMinCut is lambda * sum_s [C(s)^2 - sum_i P_i(s)^2]
 *    with C(s) = sum_i P_i(s), i.e. the sum over i != j of the Methods
 *    free energy (the literal sum over all i,j of its second term would
 *    subtract N copies of the self term).
 *  - In Max-k-SAT a repeated literal counts once and a clause holding both x
 *    and not-x is dropped (always satisfied).
 *  - Adam follows PyTorch's torch.optim.Adam (coupled L2 weight decay, eps
 *    outside the square root of the bias-corrected second moment, step count
 *    starting at 1), as the paper uses PyTorch's optimisers (Methods,
 *    "Hyperparameter tuning of different optimizers").
 *
 * Layouts: h, g, m1, m2 are [n][R] for one-logit problems and [n][R][q] for
 * Potts, node-major with the replica (then the state) index fastest.
 * Integer configurations sigma are [R][n] (replica-major), states 0..q-1; for
 * one-logit problems sigma_i = 1 means P_i (sigmoid of h_i) is the larger
 * marginal, i.e. h_i > 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Small numeric helpers                                                      */
/* ------------------------------------------------------------------------- */

/* ln(sigmoid(x)) without overflow: -log(1 + e^{-x}). */
static double log_sigmoid(double x)
{
    if (x >= 0.0) return -log1p(exp(-x));
    return x - log1p(exp(x));
}

static double sigmoid(double x)
{
    if (x >= 0.0) return 1.0 / (1.0 + exp(-x));
    double e = exp(x);
    return e / (1.0 + e);
}

/* The nearest bfloat16 value (8 significant bits, exponent range of float32,
 * ties to the even neighbour): the storage type of the marginal copy that
 * neighbours read when the copy is kept in bfloat16 (mdt = 1 below).  The
 * spacing of bfloat16 values is 2^(e-8) for |x| in [2^(e-1), 2^e), and
 * 2^-133 below 2^-126 (subnormals). */
double orc_round_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);
    int q = e - 8;
    if (q < -133) q = -133;
    return ldexp(nearbyint(ldexp(x, -q)), q);   /* nearbyint: ties to even */
}

/* ------------------------------------------------------------------------- */
/* Annealing schedules (Methods, "Different annealing schedules for the      */
/* inverse temperature").                                                     */
/*   sched 0: linear in beta, beta(0)=beta_min, beta(T-1)=beta_max           */
/*   sched 1: exponential scheduling                                         */
/*   sched 2: inverse-proportional scheduling (linear in temperature)        */
/* ------------------------------------------------------------------------- */
double orc_beta(int32_t sched, double bmin, double bmax, int32_t T, int32_t t)
{
    double x = (T > 1) ? (double)t / (double)(T - 1) : 0.0;
    if (sched == 1) return exp((log(bmax) - log(bmin)) * x + log(bmin));
    if (sched == 2) return 1.0 / ((1.0 / bmax - 1.0 / bmin) * x + 1.0 / bmin);
    return bmin + (bmax - bmin) * x;
}

/* lambda(t): constant, or increased linearly from 0 to lambda_max over the
 * annealing steps (supplementary "Demonstration of FEM solving the bMinCut
 * problem"), with the same endpoint convention as the beta schedules. */
double orc_lambda(int32_t ramp, double lam, int32_t T, int32_t t)
{
    if (!ramp) return lam;
    return (T > 1) ? lam * (double)t / (double)(T - 1) : lam;
}

/* ------------------------------------------------------------------------- */
/* MaxCut (Results, "Applications to the Maximum-Cut problem"; free energy   */
/* in Methods; explicit gradient in the supplementary "The MaxCut problem";  */
/* q = 2 reduction in "Simplification of FEM ...").                          */
/* ------------------------------------------------------------------------- */

/*
 * For every replica r: marginals P_i(+) = sigmoid(h_i), P_i(-) = 1 - P_i(+);
 *   U = -sum_{ordered (i,j)} W_ij sum_s P_i(s) [1 - P_j(s)]
 *   S = -sum_i sum_s P_i(s) ln P_i(s)
 *   g^p_i(s) = sum_j W_ij [2 P_j(s) - 1] + (ln P_i(s) + 1) / beta
 *   g^h_i    = [g^p_i(+) - g^p_i(-)] P_i(+) P_i(-)
 * g may be NULL (energies only); U, S may be NULL.
 */
int orc_maxcut_grad(int32_t n, int64_t ne, const int32_t* eu, const int32_t* ev,
                    const double* w, int32_t R, const double* h, double beta, int32_t mdt,
                    double* g, double* U, double* S)
{
    double* P = (double*)malloc(sizeof(double) * (size_t)n);
    double* Pn = (double*)malloc(sizeof(double) * (size_t)n);     /* P as neighbours read it */
    double* Wsum = (double*)malloc(sizeof(double) * (size_t)n);   /* sum_j W_ij [2P_j(+)-1] */
    if (!P || !Pn || !Wsum) { free(P); free(Pn); free(Wsum); return -2; }
    for (int32_t r = 0; r < R; ++r) {
        for (int32_t i = 0; i < n; ++i) {
            double x = h[(size_t)i * R + r];
            P[i] = sigmoid(x);
            /* bfloat16 copy: m = 2P - 1 = tanh(h/2) is what is stored */
            Pn[i] = mdt ? 0.5 * (1.0 + orc_round_bf16(tanh(0.5 * x))) : P[i];
        }
        double u_acc = 0.0, s_acc = 0.0;
        for (int32_t i = 0; i < n; ++i) Wsum[i] = 0.0;
        for (int64_t e = 0; e < ne; ++e) {
            int32_t i = eu[e], j = ev[e];
            /* the two orderings (i,j) and (j,i) of the undirected edge; the
               first index reads its own marginal, the second the stored one */
            double same_ij = P[i] * Pn[j] + (1.0 - P[i]) * (1.0 - Pn[j]);
            double same_ji = P[j] * Pn[i] + (1.0 - P[j]) * (1.0 - Pn[i]);
            u_acc += -w[e] * (1.0 - same_ij);   /* (i,j): sum_s P_i(s)[1-P_j(s)] */
            u_acc += -w[e] * (1.0 - same_ji);   /* (j,i) */
            /* sum_j W_ij [2 P_j(+) - 1] minus the same for state (-):
               [2P_j(+)-1] - [2P_j(-)-1] = 2(2P_j(+)-1) */
            Wsum[i] += w[e] * (2.0 * Pn[j] - 1.0);
            Wsum[j] += w[e] * (2.0 * Pn[i] - 1.0);
        }
        for (int32_t i = 0; i < n; ++i) {
            double x = h[(size_t)i * R + r];
            double lp = log_sigmoid(x), lm = log_sigmoid(-x);
            double pp = P[i], pm = 1.0 - P[i];
            s_acc += -(pp * lp + pm * lm);
            if (g) {
                /* state (+): sum_j W_ij[2P_j(+)-1]; state (-): sum_j W_ij[2P_j(-)-1] = -(...) */
                double gp_plus = Wsum[i] + (lp + 1.0) / beta;
                double gp_minus = -Wsum[i] + (lm + 1.0) / beta;
                /* sigmoid(x) sigmoid(-x) without cancellation */
                double pq = exp(lp + lm);
                g[(size_t)i * R + r] = (gp_plus - gp_minus) * pq;
            }
        }
        if (U) U[r] = u_acc;
        if (S) S[r] = s_acc;
    }
    free(P);
    free(Pn);
    free(Wsum);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Balanced min-cut with q Potts states (Results, "Applications to the       */
/* q-way balanced minimum cut problem"; free energy in Methods; explicit     */
/* gradient in the supplementary "The bMinCut problem"; softmax chain rule   */
/* in "The explicit gradient formulations").                                 */
/* ------------------------------------------------------------------------- */

/*
 * For every replica r: P_i(s) = softmax_s h_i(s), node weights V_i (1 when
 * V is NULL; the supplementary chip-partitioning section, where coarsened
 * nodes carry the number of nodes they group), C(s) = sum_j V_j P_j(s);
 *   U = sum_{ordered (i,j)} W_ij sum_s P_i(s)[1 - P_j(s)]
 *     + lam * sum_s [C(s)^2 - sum_i V_i^2 P_i(s)^2]
 *   S = -sum_i sum_s P_i(s) ln P_i(s)
 *   g^p_i(s) = -2 sum_j W_ij P_j(s) + 2 lam V_i [C(s) - V_i P_i(s)] + (ln P_i(s) + 1)/beta
 *   g^h_i(s) = [g^p_i(s) - sum_s' P_i(s') g^p_i(s')] P_i(s)
 */
int orc_bmincut_grad(int32_t n, int64_t ne, const int32_t* eu, const int32_t* ev,
                     const double* w, const double* V, int32_t q, double lam, int32_t R,
                     const double* h, double beta, int32_t mdt, double* g, double* U, double* S)
{
    size_t nq = (size_t)n * (size_t)q;
    double* P = (double*)malloc(sizeof(double) * nq);
    double* Pn = (double*)malloc(sizeof(double) * nq);   /* P as neighbours read it */
    double* lnP = (double*)malloc(sizeof(double) * nq);
    double* Phi = (double*)malloc(sizeof(double) * nq);
    double* C = (double*)malloc(sizeof(double) * (size_t)q);
    double* gp = (double*)malloc(sizeof(double) * (size_t)q);
    if (!P || !Pn || !lnP || !Phi || !C || !gp) {
        free(P); free(Pn); free(lnP); free(Phi); free(C); free(gp);
        return -2;
    }
    for (int32_t r = 0; r < R; ++r) {
        /* softmax per node, with the maximum subtracted before exponentiating */
        for (int32_t i = 0; i < n; ++i) {
            const double* hi = h + ((size_t)i * R + r) * q;
            double mx = hi[0];
            for (int32_t s = 1; s < q; ++s) if (hi[s] > mx) mx = hi[s];
            double Z = 0.0;
            for (int32_t s = 0; s < q; ++s) Z += exp(hi[s] - mx);
            double lz = log(Z);
            for (int32_t s = 0; s < q; ++s) {
                size_t k = (size_t)i * q + s;
                lnP[k] = hi[s] - mx - lz;
                P[k] = exp(lnP[k]);
                Pn[k] = mdt ? orc_round_bf16(P[k]) : P[k];
            }
        }
        for (int32_t s = 0; s < q; ++s) C[s] = 0.0;
        for (int32_t i = 0; i < n; ++i)
            for (int32_t s = 0; s < q; ++s) C[s] += (V ? V[i] : 1.0) * P[(size_t)i * q + s];
        for (size_t k = 0; k < nq; ++k) Phi[k] = 0.0;
        double cut_acc = 0.0;
        for (int64_t e = 0; e < ne; ++e) {
            int32_t i = eu[e], j = ev[e];
            /* ordering (i,j) reads P_i and the stored P_j, (j,i) the reverse */
            double dot_ij = 0.0, dot_ji = 0.0;
            for (int32_t s = 0; s < q; ++s) {
                dot_ij += P[(size_t)i * q + s] * Pn[(size_t)j * q + s];
                dot_ji += P[(size_t)j * q + s] * Pn[(size_t)i * q + s];
                Phi[(size_t)i * q + s] += w[e] * Pn[(size_t)j * q + s];
                Phi[(size_t)j * q + s] += w[e] * Pn[(size_t)i * q + s];
            }
            /* sum_s P_i(s)[1-P_j(s)] = 1 - P_i.P_j, once per ordering */
            cut_acc += w[e] * (1.0 - dot_ij);
            cut_acc += w[e] * (1.0 - dot_ji);
        }
        double bal = 0.0;
        for (int32_t s = 0; s < q; ++s) {
            double self = 0.0;
            for (int32_t i = 0; i < n; ++i) {
                double vp = (V ? V[i] : 1.0) * P[(size_t)i * q + s];
                self += vp * vp;
            }
            bal += C[s] * C[s] - self;
        }
        double s_acc = 0.0;
        for (size_t k = 0; k < nq; ++k) s_acc += -P[k] * lnP[k];
        if (U) U[r] = cut_acc + lam * bal;
        if (S) S[r] = s_acc;
        if (g) {
            for (int32_t i = 0; i < n; ++i) {
                double avg = 0.0;
                for (int32_t s = 0; s < q; ++s) {
                    size_t k = (size_t)i * q + s;
                    double vi = V ? V[i] : 1.0;
                    gp[s] = -2.0 * Phi[k] + 2.0 * lam * vi * (C[s] - vi * P[k]) + (lnP[k] + 1.0) / beta;
                    avg += P[k] * gp[s];
                }
                for (int32_t s = 0; s < q; ++s) {
                    size_t k = (size_t)i * q + s;
                    g[((size_t)i * R + r) * q + s] = (gp[s] - avg) * P[k];
                }
            }
        }
    }
    free(P); free(Pn); free(lnP); free(Phi); free(C); free(gp);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Max-k-SAT (Results, "Application to the Max k-SAT problem"; free energy   */
/* in Methods; explicit gradient in the supplementary "The MaxSAT problem",  */
/* whose product index is read as P_k(W_mk), the literal of variable k in    */
/* clause m).                                                                 */
/* ------------------------------------------------------------------------- */

/* Canonical clause: distinct variables with their literal signs. Returns the
 * number of distinct variables, or -1 for a clause holding x and not-x. */
static int canon_clause(const int32_t* lit, int64_t len, int32_t* var, int32_t* pos)
{
    int k = 0;
    for (int64_t a = 0; a < len; ++a) {
        int32_t L = lit[a];
        int32_t x = (L > 0 ? L : -L) - 1;
        int32_t sp = L > 0;
        int seen = 0;
        for (int b = 0; b < k; ++b) {
            if (var[b] == x) {
                if (pos[b] != sp) return -1; /* tautology */
                seen = 1;
            }
        }
        if (!seen) { var[k] = x; pos[k] = sp; ++k; }
    }
    return k;
}

/*
 * W_mi = 1 for a positive literal; P_i(1) = sigmoid(h_i).  For every replica:
 *   U = sum_m prod_{i in dm} [1 - P_i(W_mi)]
 *   S = -sum_i sum_s P_i(s) ln P_i(s)
 *   g^p_i(s) = -sum_m delta(s, W_mi) prod_{k in dm, k != i} [1 - P_k(W_mk)]
 *              + (ln P_i(s) + 1)/beta
 *   g^h_i = [g^p_i(1) - g^p_i(0)] P_i(1) P_i(0)
 */
int orc_maxsat_grad(int32_t n, int64_t M, const int64_t* off, const int32_t* lits,
                    int32_t R, const double* h, double beta, int32_t mdt, double* g, double* U, double* S)
{
    int64_t kmax = 0;
    for (int64_t m = 0; m < M; ++m) if (off[m + 1] - off[m] > kmax) kmax = off[m + 1] - off[m];
    int32_t* var = (int32_t*)malloc(sizeof(int32_t) * (size_t)(kmax + 1));
    int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(kmax + 1));
    double* ufalse = (double*)malloc(sizeof(double) * (size_t)(kmax + 1));
    double* ustore = (double*)malloc(sizeof(double) * (size_t)(kmax + 1));   /* as other literals read it */
    double* gp1 = (double*)malloc(sizeof(double) * (size_t)n);  /* energy part of g^p_i(1) */
    double* gp0 = (double*)malloc(sizeof(double) * (size_t)n);  /* energy part of g^p_i(0) */
    if (!var || !pos || !ufalse || !ustore || !gp1 || !gp0) {
        free(var); free(pos); free(ufalse); free(ustore); free(gp1); free(gp0);
        return -2;
    }
    for (int32_t r = 0; r < R; ++r) {
        for (int32_t i = 0; i < n; ++i) { gp1[i] = 0.0; gp0[i] = 0.0; }
        double u_acc = 0.0;
        for (int64_t m = 0; m < M; ++m) {
            int k = canon_clause(lits + off[m], off[m + 1] - off[m], var, pos);
            if (k < 0) continue;
            for (int a = 0; a < k; ++a) {
                double x = h[(size_t)var[a] * R + r];
                double p1 = sigmoid(x);
                /* 1 - P_i(W_mi): the probability that this literal is false */
                ufalse[a] = pos[a] ? 1.0 - p1 : p1;
                ustore[a] = ufalse[a];
                if (mdt) {
                    /* bfloat16 copy: the smaller marginal min(P, 1 - P) is
                       stored, the larger one is 1 minus it */
                    double small = orc_round_bf16(sigmoid(-fabs(x)));
                    int literal_likely = (x > 0.0) == (pos[a] != 0);
                    ustore[a] = literal_likely ? small : 1.0 - small;
                }
            }
            /* the clause's energy as its first literal evaluates it: its own
               marginal and the others' stored ones */
            double prod = ufalse[0];
            for (int a = 1; a < k; ++a) prod *= ustore[a];
            u_acc += prod;
            for (int a = 0; a < k; ++a) {
                double cav = 1.0;
                for (int b = 0; b < k; ++b) if (b != a) cav *= ustore[b];
                if (pos[a]) gp1[var[a]] -= cav; else gp0[var[a]] -= cav;
            }
        }
        double s_acc = 0.0;
        for (int32_t i = 0; i < n; ++i) {
            double x = h[(size_t)i * R + r];
            double l1 = log_sigmoid(x), l0 = log_sigmoid(-x);
            double p1 = exp(l1), p0 = exp(l0);
            s_acc += -(p1 * l1 + p0 * l0);
            if (g) {
                double a1 = gp1[i] + (l1 + 1.0) / beta;
                double a0 = gp0[i] + (l0 + 1.0) / beta;
                g[(size_t)i * R + r] = (a1 - a0) * exp(l1 + l0);
            }
        }
        if (U) U[r] = u_acc;
        if (S) S[r] = s_acc;
    }
    free(var); free(pos); free(ufalse); free(ustore); free(gp1); free(gp0);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Manipulated gradients (supplementary "The explicit gradient formulations" */
/* and "The explicit gradients and manipulated gradients for the             */
/* benchmarking problems").  The gradient with respect to P is replaced by a */
/* modified one, ghat, which is not the derivative of any free energy, and   */
/* the softmax chain rule gives                                              */
/*   g^h_i(s) = gamma [ghat_i(s) - sum_s' P_i(s') ghat_i(s')] P_i(s).        */
/* The neighbours enter only through one-hot vectors e_j of their current    */
/* read-out (the discretisation), with per-node normalisation factors.       */
/* One-hot read-out: the state of largest field, ties to the lowest state;   */
/* for one logit, state (+) iff h > 0.  A node without incident weight gets  */
/* normalisation factor 0 (its sums are empty).                              */
/* ------------------------------------------------------------------------- */

/*
 * MaxCut, states (+) and (-), P_i(+) = sigmoid(h_i):
 *   ghat_i(s) = c_i sum_j W_ij e_j(s) + (ln P_i(s) + 1) / beta,
 *   c_i = 1 / sum_j |W_ij|,
 *   g^h_i = g^h_i(+) of the chain rule above with q = 2.
 */
int orc_maxcut_grad_manip(int32_t n, int64_t ne, const int32_t* eu, const int32_t* ev,
                          const double* w, int32_t R, const double* h, double beta,
                          double gamma, double* g)
{
    double* L1 = (double*)calloc((size_t)n, sizeof(double));     /* sum_j |W_ij| */
    double* Eplus = (double*)malloc(sizeof(double) * (size_t)n); /* sum_j W_ij e_j(+) */
    double* Eminus = (double*)malloc(sizeof(double) * (size_t)n);
    if (!L1 || !Eplus || !Eminus) { free(L1); free(Eplus); free(Eminus); return -2; }
    for (int64_t e = 0; e < ne; ++e) {
        L1[eu[e]] += fabs(w[e]);
        L1[ev[e]] += fabs(w[e]);
    }
    for (int32_t r = 0; r < R; ++r) {
        for (int32_t i = 0; i < n; ++i) Eplus[i] = Eminus[i] = 0.0;
        for (int64_t e = 0; e < ne; ++e) {
            int32_t i = eu[e], j = ev[e];
            /* one-hot read-out of each endpoint: (+) iff its field is positive */
            int plus_j = h[(size_t)j * R + r] > 0.0, plus_i = h[(size_t)i * R + r] > 0.0;
            if (plus_j) Eplus[i] += w[e]; else Eminus[i] += w[e];
            if (plus_i) Eplus[j] += w[e]; else Eminus[j] += w[e];
        }
        for (int32_t i = 0; i < n; ++i) {
            double x = h[(size_t)i * R + r];
            double c = L1[i] > 0.0 ? 1.0 / L1[i] : 0.0;
            double lp = log_sigmoid(x), lm = log_sigmoid(-x);
            double pp = exp(lp), pm = exp(lm);
            double gh_plus = c * Eplus[i] + (lp + 1.0) / beta;
            double gh_minus = c * Eminus[i] + (lm + 1.0) / beta;
            double avg = pp * gh_plus + pm * gh_minus;
            g[(size_t)i * R + r] = gamma * (gh_plus - avg) * pp;
        }
    }
    free(L1); free(Eplus); free(Eminus);
    return 0;
}

/*
 * bMinCut, q states, P_i = softmax h_i, weights W_ij > 0, lam = lambda(t),
 * node weights V_i (1 when V is NULL):
 *   ghat_i(s) = -c^f_i sum_j W_ij e_j(s) + lam c^a_i V_i [sum_j V_j e_j(s) - V_i e_i(s)]
 *               + (ln P_i(s) + 1) / beta,
 *   c^f_i = q / sum_j W_ij,  c^a_i = q / sqrt(sum_j W_ij),
 * where sum_j V_j e_j(s) runs over all nodes (the weight of group s in the
 * current read-out).
 */
int orc_bmincut_grad_manip(int32_t n, int64_t ne, const int32_t* eu, const int32_t* ev,
                           const double* w, const double* V, int32_t q, double lam, int32_t R,
                           const double* h, double beta, double gamma, double* g)
{
    size_t nq = (size_t)n * (size_t)q;
    double* D = (double*)calloc((size_t)n, sizeof(double));      /* sum_j W_ij */
    int32_t* e1 = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);  /* one-hot as a state index */
    double* F = (double*)malloc(sizeof(double) * nq);            /* sum_j W_ij e_j(s) */
    double* cnt = (double*)malloc(sizeof(double) * (size_t)q);   /* sum_j e_j(s) */
    double* lnP = (double*)malloc(sizeof(double) * (size_t)q);
    double* gh = (double*)malloc(sizeof(double) * (size_t)q);
    if (!D || !e1 || !F || !cnt || !lnP || !gh) {
        free(D); free(e1); free(F); free(cnt); free(lnP); free(gh);
        return -2;
    }
    for (int64_t e = 0; e < ne; ++e) {
        D[eu[e]] += w[e];
        D[ev[e]] += w[e];
    }
    for (int32_t r = 0; r < R; ++r) {
        for (int32_t s = 0; s < q; ++s) cnt[s] = 0.0;
        for (int32_t i = 0; i < n; ++i) {
            const double* hi = h + ((size_t)i * R + r) * q;
            int32_t best = 0;
            for (int32_t s = 1; s < q; ++s) if (hi[s] > hi[best]) best = s;
            e1[i] = best;
            cnt[best] += V ? V[i] : 1.0;
        }
        for (size_t k = 0; k < nq; ++k) F[k] = 0.0;
        for (int64_t e = 0; e < ne; ++e) {
            int32_t i = eu[e], j = ev[e];
            F[(size_t)i * q + e1[j]] += w[e];
            F[(size_t)j * q + e1[i]] += w[e];
        }
        for (int32_t i = 0; i < n; ++i) {
            const double* hi = h + ((size_t)i * R + r) * q;
            double mx = hi[0];
            for (int32_t s = 1; s < q; ++s) if (hi[s] > mx) mx = hi[s];
            double Z = 0.0;
            for (int32_t s = 0; s < q; ++s) Z += exp(hi[s] - mx);
            double lz = log(Z);
            for (int32_t s = 0; s < q; ++s) lnP[s] = hi[s] - mx - lz;
            double cf = D[i] > 0.0 ? (double)q / D[i] : 0.0;
            double ca = D[i] > 0.0 ? (double)q / sqrt(D[i]) : 0.0;
            double avg = 0.0;
            for (int32_t s = 0; s < q; ++s) {
                double vi = V ? V[i] : 1.0;
                double own = (e1[i] == s) ? vi : 0.0;
                gh[s] = -cf * F[(size_t)i * q + s] + lam * ca * vi * (cnt[s] - own) + (lnP[s] + 1.0) / beta;
                avg += exp(lnP[s]) * gh[s];
            }
            for (int32_t s = 0; s < q; ++s)
                g[((size_t)i * R + r) * q + s] = gamma * (gh[s] - avg) * exp(lnP[s]);
        }
    }
    free(D); free(e1); free(F); free(cnt); free(lnP); free(gh);
    return 0;
}

/*
 * Max-k-SAT: the paper leaves the gradient unmodified (ghat = g^p), so the
 * manipulated form is gamma times the explicit gradient.
 */
int orc_maxsat_grad_manip(int32_t n, int64_t M, const int64_t* off, const int32_t* lits,
                          int32_t R, const double* h, double beta, double gamma, double* g)
{
    int rc = orc_maxsat_grad(n, M, off, lits, R, h, beta, 0, g, NULL, NULL);
    if (rc) return rc;
    for (size_t k = 0; k < (size_t)n * (size_t)R; ++k) g[k] *= gamma;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Adam (Kingma & Ba), PyTorch semantics: n_step counts from 1.              */
/* ------------------------------------------------------------------------- */
void orc_adam(int64_t count, const double* g_in, double* h, double* m1, double* m2,
              double lr, double b1, double b2, double eps, double wd, int64_t n_step)
{
    double bc1 = 1.0 - pow(b1, (double)n_step);
    double bc2 = 1.0 - pow(b2, (double)n_step);
    for (int64_t k = 0; k < count; ++k) {
        double g = g_in[k] + wd * h[k];
        m1[k] = b1 * m1[k] + (1.0 - b1) * g;
        m2[k] = b2 * m2[k] + (1.0 - b2) * g * g;
        double mhat = m1[k] / bc1;
        double vhat = m2[k] / bc2;
        h[k] -= lr * mhat / (sqrt(vhat) + eps);
    }
}

/* RMSprop, PyTorch semantics (not centred): m2 = square average, m1 = the
 * momentum buffer (used when momentum > 0).  The paper tunes lr, alpha,
 * momentum and weight decay (Methods, "Hyperparameter tuning"). */
void orc_rmsprop(int64_t count, const double* g_in, double* h, double* m1, double* m2,
                 double lr, double alpha, double eps, double wd, double momentum)
{
    for (int64_t k = 0; k < count; ++k) {
        double g = g_in[k] + wd * h[k];
        m2[k] = alpha * m2[k] + (1.0 - alpha) * g * g;
        double avg = sqrt(m2[k]) + eps;
        if (momentum > 0.0) {
            m1[k] = momentum * m1[k] + g / avg;
            h[k] -= lr * m1[k];
        } else {
            h[k] -= lr * g / avg;
        }
    }
}

/* SGD, PyTorch semantics: with momentum, the buffer starts as the first
 * gradient and then follows buf = momentum buf + (1 - dampening) g. */
void orc_sgd(int64_t count, const double* g_in, double* h, double* m1, double lr, double wd,
             double momentum, double dampening, int64_t n_step)
{
    for (int64_t k = 0; k < count; ++k) {
        double g = g_in[k] + wd * h[k];
        if (momentum != 0.0) {
            m1[k] = (n_step == 1) ? g : momentum * m1[k] + (1.0 - dampening) * g;
            g = m1[k];
        }
        h[k] -= lr * g;
    }
}

/* ------------------------------------------------------------------------- */
/* Read-out (Results, "Free-Energy Machine": argmax of each replica's         */
/* marginals, then the replica of lowest energy).                             */
/* ------------------------------------------------------------------------- */

/* sigma[r][i] = argmax_s P_i(s) with ties to the lowest state index.  For
 * q == 1 (one logit) the two states are 0 (P = 1 - sigmoid(h)) and 1
 * (P = sigmoid(h)), so sigma = 1 iff h > 0. */
void orc_round(int32_t n, int32_t R, int32_t q, const double* h, int32_t* sigma)
{
    for (int32_t r = 0; r < R; ++r)
        for (int32_t i = 0; i < n; ++i) {
            if (q == 1) {
                sigma[(size_t)r * n + i] = h[(size_t)i * R + r] > 0.0 ? 1 : 0;
            } else {
                const double* hi = h + ((size_t)i * R + r) * q;
                int32_t best = 0;
                for (int32_t s = 1; s < q; ++s) if (hi[s] > hi[best]) best = s;
                sigma[(size_t)r * n + i] = best;
            }
        }
}

/* Cut value sum over undirected edges of W_ij [sigma_i != sigma_j] (each edge
 * once, the listing's cut(W, s)/2).  Works for any number of states. */
void orc_cut(int32_t n, int64_t ne, const int32_t* eu, const int32_t* ev, const double* w,
             int32_t R, const int32_t* sigma, double* cut)
{
    for (int32_t r = 0; r < R; ++r) {
        const int32_t* sg = sigma + (size_t)r * n;
        double c = 0.0;
        for (int64_t e = 0; e < ne; ++e)
            if (sg[eu[e]] != sg[ev[e]]) c += w[e];
        cut[r] = c;
    }
}

/* Group sizes |Pi_s| = #{i : sigma_i = s} per replica, [R][q]. */
void orc_group_sizes(int32_t n, int32_t q, int32_t R, const int32_t* sigma, const int32_t* V, int64_t* sizes)
{
    for (int32_t r = 0; r < R; ++r) {
        for (int32_t s = 0; s < q; ++s) sizes[(size_t)r * q + s] = 0;
        for (int32_t i = 0; i < n; ++i) sizes[(size_t)r * q + sigma[(size_t)r * n + i]] += V ? V[i] : 1;
    }
}

/* Number of unsatisfied clauses (every literal false) per replica; sigma is
 * 0/1 per variable.  A tautological clause is always satisfied. */
void orc_unsat(int32_t n, int64_t M, const int64_t* off, const int32_t* lits, int32_t R,
               const int32_t* sigma, int64_t* unsat)
{
    for (int32_t r = 0; r < R; ++r) {
        const int32_t* sg = sigma + (size_t)r * n;
        int64_t c = 0;
        for (int64_t m = 0; m < M; ++m) {
            int sat = 0;
            for (int64_t a = off[m]; a < off[m + 1]; ++a) {
                int32_t L = lits[a];
                int32_t x = (L > 0 ? L : -L) - 1;
                if ((L > 0 && sg[x] == 1) || (L < 0 && sg[x] == 0)) { sat = 1; break; }
            }
            if (!sat) ++c;
        }
        unsat[r] = c;
    }
}

/* ------------------------------------------------------------------------- */
/* The annealing loop (Methods listing and Fig. 2 workflow): for each step    */
/* t, beta = beta(t), gradient of F at h(t), Adam update with step count     */
/* t+1.  kind 0 = MaxCut, 1 = bMinCut, 2 = Max-k-SAT.  Runs steps t0 ..      */
/* t0+n_steps-1 of a T-step schedule.  Optional histories (NULL to skip):    */
/* g_hist [n_steps][vals], U_hist/S_hist [n_steps][R].                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t kind, n, q, R, T, sched, lam_ramp;
    int64_t ne;             /* edges (graphs) or clauses (SAT) */
    const int32_t* eu;      /* graphs */
    const int32_t* ev;
    const double* w;
    const int64_t* off;     /* SAT */
    const int32_t* lits;
    double beta_min, beta_max, lam, lr, b1, b2, eps, wd;
    int32_t opt;            /* 0 Adam, 1 RMSprop, 2 SGD */
    double momentum, rms_alpha, dampening;
    int32_t manip;          /* 1: manipulated gradients (no energies) */
    double gamma;           /* gamma_grad of the manipulated form */
    const double* nw;       /* bMinCut node weights (NULL: all 1) */
    int32_t mdt;            /* 1: neighbours read a bfloat16 copy of the marginals */
} orc_problem;

int orc_run(const orc_problem* pb, int32_t t0, int32_t n_steps, double* h, double* m1,
            double* m2, double* g_hist, double* U_hist, double* S_hist)
{
    int32_t Q = pb->kind == 1 ? pb->q : 1;
    size_t vals = (size_t)pb->n * (size_t)pb->R * (size_t)Q;
    double* g = (double*)malloc(sizeof(double) * vals);
    if (!g) return -2;
    for (int32_t k = 0; k < n_steps; ++k) {
        int32_t t = t0 + k;
        double beta = orc_beta(pb->sched, pb->beta_min, pb->beta_max, pb->T, t);
        double* U = U_hist ? U_hist + (size_t)k * pb->R : NULL;
        double* S = S_hist ? S_hist + (size_t)k * pb->R : NULL;
        int rc;
        if (pb->manip && pb->kind == 0)
            rc = orc_maxcut_grad_manip(pb->n, pb->ne, pb->eu, pb->ev, pb->w, pb->R, h, beta, pb->gamma, g);
        else if (pb->manip && pb->kind == 1)
            rc = orc_bmincut_grad_manip(pb->n, pb->ne, pb->eu, pb->ev, pb->w, pb->nw, pb->q,
                                        orc_lambda(pb->lam_ramp, pb->lam, pb->T, t), pb->R, h, beta,
                                        pb->gamma, g);
        else if (pb->manip)
            rc = orc_maxsat_grad_manip(pb->n, pb->ne, pb->off, pb->lits, pb->R, h, beta, pb->gamma, g);
        else if (pb->kind == 0)
            rc = orc_maxcut_grad(pb->n, pb->ne, pb->eu, pb->ev, pb->w, pb->R, h, beta, pb->mdt, g, U, S);
        else if (pb->kind == 1)
            rc = orc_bmincut_grad(pb->n, pb->ne, pb->eu, pb->ev, pb->w, pb->nw, pb->q,
                                  orc_lambda(pb->lam_ramp, pb->lam, pb->T, t), pb->R, h, beta, pb->mdt, g, U, S);
        else
            rc = orc_maxsat_grad(pb->n, pb->ne, pb->off, pb->lits, pb->R, h, beta, pb->mdt, g, U, S);
        if (rc) { free(g); return rc; }
        if (g_hist) memcpy(g_hist + (size_t)k * vals, g, sizeof(double) * vals);
        if (pb->opt == 1)
            orc_rmsprop((int64_t)vals, g, h, m1, m2, pb->lr, pb->rms_alpha, pb->eps, pb->wd, pb->momentum);
        else if (pb->opt == 2)
            orc_sgd((int64_t)vals, g, h, m1, pb->lr, pb->wd, pb->momentum, pb->dampening, (int64_t)t + 1);
        else
            orc_adam((int64_t)vals, g, h, m1, m2, pb->lr, pb->b1, pb->b2, pb->eps, pb->wd, (int64_t)t + 1);
    }
    free(g);
    return 0;
}
