/*
 * Plain FP64 CPU oracle for syndrome-form flooding sum-product decoding of
 * quasi-cyclic LDPC codes.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP decoder is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code with the HIP decoder.
 *
 * What it follows:
 *  - QC lifting, Sec. III-C: every non-zero base entry is a Z x Z circulant
 *    permutation; with the 0-based shift s (the paper's I_i has s = i - 1),
 *    row a of the block has its 1 in column (a + s) mod Z.
 *  - Algorithm 1 (Sec. III-D), Steps 1-4, in the order printed, on an
 *    explicitly expanded parity-check matrix, in double precision:
 *      Step 1  L_vc <- Q_v for every edge;
 *      Step 2  check update in the Phi domain, Phi(x) = -ln tanh(x/2);
 *      Step 3  variable update (extrinsic L_vc and posterior L_v);
 *      Step 4  hard decision (L_v >= 0 -> 0) and the parity check.
 *  - Syndrome form (the Slepian-Wolf view of reverse reconciliation,
 *    Sec. II-C.4): each check c carries a target bit s_c; its outgoing
 *    messages are multiplied by (-1)^{s_c} and decoding stops when
 *    H x = s.  With s = 0 this is Algorithm 1 exactly.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *  - the parity check also runs once before the first iteration, so a frame
 *    whose channel decisions already satisfy H x = s reports 0 iterations;
 *  - sgn(0) = +1 inside the sign products;
 *  - the argument of every Phi evaluation is clamped to [1e-7, 30];
 *  - Phi is evaluated as log1p(2 / expm1(x)), which equals -ln tanh(x/2)
 *    without cancellation for large x;
 *  - check_from delays the parity check to iterations t >= check_from (the
 *    paper's early-termination lookup table, Sec. IV-A); 0 = every iteration.
 *
 * Parity pins: see the oracle pin tests (brute-force MAP marginals on
 * cycle-free codes, closed-form check rules, noiseless inputs, coset
 * equivariance, the H x = s invariant).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHI_LO 1e-7
#define PHI_HI 30.0

typedef struct {
    int mb, nb, Z;
    int n, m, E;
    int *edge_var;      /* [E] variable of each edge                */
    int *edge_chk;      /* [E] check of each edge                   */
    int *chk_ptr;       /* [m+1] edges of check c: chk_edges[ptr..] */
    int *chk_edges;     /* [E]                                      */
    int *var_ptr;       /* [n+1] edges of variable v                */
    int *var_edges;     /* [E]                                      */
} oracle_code;

/* Phi(x) = -ln tanh(x/2) = log1p(2/expm1(x)), on the clamped argument. */
double oracle_phi(double x)
{
    if (x < PHI_LO) x = PHI_LO;
    if (x > PHI_HI) x = PHI_HI;
    return log1p(2.0 / expm1(x));
}

void oracle_code_free(oracle_code *c)
{
    if (!c) return;
    free(c->edge_var); free(c->edge_chk);
    free(c->chk_ptr); free(c->chk_edges);
    free(c->var_ptr); free(c->var_edges);
    free(c);
}

/* Expand the base matrix (mb x nb, row-major; -1 = zero block, else shift in
 * [0, Z)) into an explicit edge list with check-major and variable-major
 * adjacency.  Returns NULL on a bad argument or allocation failure. */
oracle_code *oracle_code_build(int mb, int nb, const int32_t *base, int Z)
{
    if (mb < 1 || nb < 1 || Z < 1 || !base) return NULL;
    int blocks = 0;
    for (int i = 0; i < mb * nb; i++) {
        if (base[i] >= Z || base[i] < -1) return NULL;
        if (base[i] >= 0) blocks++;
    }
    oracle_code *c = (oracle_code *)calloc(1, sizeof(oracle_code));
    if (!c) return NULL;
    c->mb = mb; c->nb = nb; c->Z = Z;
    c->n = nb * Z; c->m = mb * Z; c->E = blocks * Z;
    size_t E = (size_t)c->E;
    c->edge_var = (int *)malloc(E * sizeof(int) + 1);
    c->edge_chk = (int *)malloc(E * sizeof(int) + 1);
    c->chk_edges = (int *)malloc(E * sizeof(int) + 1);
    c->var_edges = (int *)malloc(E * sizeof(int) + 1);
    c->chk_ptr = (int *)calloc((size_t)c->m + 1, sizeof(int));
    c->var_ptr = (int *)calloc((size_t)c->n + 1, sizeof(int));
    if (!c->edge_var || !c->edge_chk || !c->chk_edges || !c->var_edges ||
        !c->chk_ptr || !c->var_ptr) {
        oracle_code_free(c);
        return NULL;
    }
    /* H(r*Z + a, col*Z + (a + s) mod Z) = 1 for every block and every a. */
    int e = 0;
    for (int r = 0; r < mb; r++)
        for (int col = 0; col < nb; col++) {
            int s = base[r * nb + col];
            if (s < 0) continue;
            for (int a = 0; a < Z; a++) {
                c->edge_chk[e] = r * Z + a;
                c->edge_var[e] = col * Z + (a + s) % Z;
                e++;
            }
        }
    /* adjacency lists, each in increasing edge order */
    for (e = 0; e < c->E; e++) {
        c->chk_ptr[c->edge_chk[e] + 1]++;
        c->var_ptr[c->edge_var[e] + 1]++;
    }
    for (int i = 0; i < c->m; i++) c->chk_ptr[i + 1] += c->chk_ptr[i];
    for (int i = 0; i < c->n; i++) c->var_ptr[i + 1] += c->var_ptr[i];
    int *fill_c = (int *)calloc((size_t)c->m + 1, sizeof(int));
    int *fill_v = (int *)calloc((size_t)c->n + 1, sizeof(int));
    if (!fill_c || !fill_v) {
        free(fill_c); free(fill_v);
        oracle_code_free(c);
        return NULL;
    }
    for (e = 0; e < c->E; e++) {
        int ch = c->edge_chk[e], v = c->edge_var[e];
        c->chk_edges[c->chk_ptr[ch] + fill_c[ch]++] = e;
        c->var_edges[c->var_ptr[v] + fill_v[v]++] = e;
    }
    free(fill_c); free(fill_v);
    return c;
}

int oracle_code_n(const oracle_code *c) { return c->n; }
int oracle_code_m(const oracle_code *c) { return c->m; }
int oracle_code_edges(const oracle_code *c) { return c->E; }

/* Copy the expanded edge list out: check and variable of every edge. */
void oracle_code_edge_list(const oracle_code *c, int32_t *chk, int32_t *var)
{
    for (int e = 0; e < c->E; e++) { chk[e] = c->edge_chk[e]; var[e] = c->edge_var[e]; }
}

/* s = H x (mod 2) for one word of n bits (values 0/1). */
void oracle_syndrome(const oracle_code *c, const uint8_t *x, uint8_t *s)
{
    for (int ch = 0; ch < c->m; ch++) {
        int p = 0;
        for (int k = c->chk_ptr[ch]; k < c->chk_ptr[ch + 1]; k++)
            p ^= x[c->edge_var[c->chk_edges[k]]] & 1;
        s[ch] = (uint8_t)p;
    }
}

static int satisfies(const oracle_code *c, const uint8_t *x, const uint8_t *s)
{
    for (int ch = 0; ch < c->m; ch++) {
        int p = s[ch] & 1;
        for (int k = c->chk_ptr[ch]; k < c->chk_ptr[ch + 1]; k++)
            p ^= x[c->edge_var[c->chk_edges[k]]] & 1;
        if (p) return 0;
    }
    return 1;
}

/*
 * Decode one frame.
 *   Q        [n] channel LLRs (ln P(0)/P(1)), double
 *   s        [m] syndrome bits, 0/1
 *   max_iters     T >= 0
 *   early_stop    1: stop at the first checked iteration with H x = s
 *   check_from    first iteration at which the check runs (0 = from the start)
 *   bits     [n] out: hard decisions x_v = [L_v < 0]
 *   L        [n] out: posterior L_v at exit (may be NULL)
 *   iters    out: iterations completed at exit
 * Returns 1 if H x = s at exit, 0 if not, -1 on allocation failure.
 */
int oracle_decode(const oracle_code *c, const double *Q, const uint8_t *s,
                  int max_iters, int early_stop, int check_from,
                  uint8_t *bits, double *L, int *iters)
{
    const int n = c->n, m = c->m, E = c->E;
    double *Lvc = (double *)malloc((size_t)E * sizeof(double) + 1);  /* VN-to-CN messages */
    double *mcv = (double *)malloc((size_t)E * sizeof(double) + 1);  /* CN-to-VN messages */
    double *Lv = (double *)malloc((size_t)n * sizeof(double) + 1);   /* posteriors        */
    int maxdeg = 1;
    for (int ch = 0; ch < m; ch++) {
        int d = c->chk_ptr[ch + 1] - c->chk_ptr[ch];
        if (d > maxdeg) maxdeg = d;
    }
    double *phin = (double *)malloc((size_t)maxdeg * sizeof(double));
    int *neg = (int *)malloc((size_t)maxdeg * sizeof(int));
    if (!Lvc || !mcv || !Lv || !phin || !neg) {
        free(Lvc); free(mcv); free(Lv); free(phin); free(neg);
        return -1;
    }

    /* Step 1: L_vc(0) = Q_v on every edge; the t = 0 decision uses L_v = Q_v. */
    for (int e = 0; e < E; e++) Lvc[e] = Q[c->edge_var[e]];
    for (int v = 0; v < n; v++) {
        Lv[v] = Q[v];
        bits[v] = (uint8_t)(Lv[v] < 0.0);
    }
    int t = 0;
    int ok = satisfies(c, bits, s);
    if (!(early_stop && check_from <= 0 && ok)) {
        for (t = 1; t <= max_iters; t++) {
            /* Step 2: check update. For edge k of check ch, combine the other
             * edges' inputs: sign = (-1)^{s_ch} * prod sgn(L_v'c),
             * magnitude = Phi( sum Phi(|L_v'c|) ). */
            for (int ch = 0; ch < m; ch++) {
                int b = c->chk_ptr[ch], d = c->chk_ptr[ch + 1] - b;
                for (int k = 0; k < d; k++) {
                    double x = Lvc[c->chk_edges[b + k]];
                    neg[k] = x < 0.0;
                    phin[k] = oracle_phi(fabs(x));
                }
                for (int k = 0; k < d; k++) {
                    double sum = 0.0;
                    int par = s[ch] & 1;
                    for (int j = 0; j < d; j++) {
                        if (j == k) continue;
                        sum += phin[j];
                        par ^= neg[j];
                    }
                    double mag = oracle_phi(sum);
                    mcv[c->chk_edges[b + k]] = par ? -mag : mag;
                }
            }
            /* Step 3: variable update. L_vc = Q_v + sum over the other checks,
             * L_v = Q_v + sum over all checks. */
            for (int v = 0; v < n; v++) {
                int b = c->var_ptr[v], d = c->var_ptr[v + 1] - b;
                double tot = Q[v];
                for (int k = 0; k < d; k++) tot += mcv[c->var_edges[b + k]];
                Lv[v] = tot;
                for (int k = 0; k < d; k++) {
                    double ext = Q[v];
                    for (int j = 0; j < d; j++)
                        if (j != k) ext += mcv[c->var_edges[b + j]];
                    Lvc[c->var_edges[b + k]] = ext;
                }
            }
            /* Step 4: hard decision, then the parity check. */
            for (int v = 0; v < n; v++) bits[v] = (uint8_t)(Lv[v] < 0.0);
            ok = satisfies(c, bits, s);
            if (early_stop && t >= check_from && ok) break;
        }
        if (t > max_iters) t = max_iters;
    }
    if (L) memcpy(L, Lv, (size_t)n * sizeof(double));
    *iters = t;
    free(Lvc); free(mcv); free(Lv); free(phin); free(neg);
    return ok;
}
