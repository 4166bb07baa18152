/*
 * CPU oracle for syndrome-based normalized min-sum decoding.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the decoder library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the device path.
 *
 * Every routine is a plain, slow, scalar restatement of the method of
 * "GPU-Accelerated Syndrome Decoding for Quantum LDPC Codes below the 63 us
 * Latency Threshold", Section 2, Algorithm 1 (min-sum for syndrome-based
 * decoding), with these readings of points the paper leaves open:
 *
 *  - the syndrome bit s_m enters the check-node sign as (-1)^{s_m};
 *  - sg(x) = -1 iff x < 0, so sg(-0.0) = +1, matching the decision rule
 *    e_n = 1 iff Q_n < 0;
 *  - the prior gamma_n is an input (the paper initialises it to 1; decoding
 *    is positively homogeneous in gamma, so a uniform gamma gives the same
 *    hard decisions as gamma = 1);
 *  - stopping: run at most I_max iterations; after iteration k's decision,
 *    stop iff H e^(k) = s (when early stopping is on).  Without convergence
 *    the outputs are those of iteration I_max;
 *  - floating point: every sum is taken left to right starting from gamma_n
 *    in increasing check index, alpha * min is rounded once, and no fused
 *    multiply-add is allowed (built with -ffp-contract=off);
 *  - integer formats (the paper's reduced-precision data types, Section 3,
 *    Table 1: 8- and 16-bit integers): messages saturate symmetrically to
 *    [-qmax, qmax] (127, or 32767), priors are signed fixed point (Q4 in
 *    int8, Q8 in int16), alpha = num / 2^sh is applied to the magnitude and
 *    rounded down before the sign, and every sum is exact in int32.
 *
 * Inside a step the oracle uses the plain definition: for every output edge
 * the excluded minimum, excluded sign product and excluded sum are formed
 * by an explicit loop over the other edges, O(d^2) per node.
 *
 * The parity-check matrix arrives dense (m x n bytes, nonzero = edge); the
 * oracle derives its own adjacency: S_v(m) in increasing column order and
 * S_c(n) in increasing row order.  Edge index e is the position of (m, n)
 * in row-major order, which indexes the per-edge neural weights.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int m, n, nnz;
    int *row_ptr;   /* m + 1 */
    int *col;       /* nnz: column of edge e */
    int *vn_ptr;    /* n + 1 */
    int *vn_edge;   /* nnz: edges of variable n in increasing row order */
    int *vn_row;    /* nnz: the row of that edge */
} graph_t;

static int graph_build(graph_t *g, int m, int n, const uint8_t *H) {
    memset(g, 0, sizeof(*g));
    g->m = m;
    g->n = n;
    int nnz = 0;
    for (long i = 0; i < (long)m * n; i++) nnz += H[i] != 0;
    g->nnz = nnz;
    g->row_ptr = calloc((size_t)m + 1, sizeof(int));
    g->col = calloc((size_t)nnz + 1, sizeof(int));
    g->vn_ptr = calloc((size_t)n + 1, sizeof(int));
    g->vn_edge = calloc((size_t)nnz + 1, sizeof(int));
    g->vn_row = calloc((size_t)nnz + 1, sizeof(int));
    if (!g->row_ptr || !g->col || !g->vn_ptr || !g->vn_edge || !g->vn_row) return -1;
    int e = 0;
    for (int r = 0; r < m; r++) {
        g->row_ptr[r] = e;
        for (int c = 0; c < n; c++)
            if (H[(long)r * n + c]) g->col[e++] = c;
    }
    g->row_ptr[m] = e;
    int k = 0;
    for (int c = 0; c < n; c++) {
        g->vn_ptr[c] = k;
        for (int r = 0; r < m; r++)
            if (H[(long)r * n + c]) {
                /* find the edge index of (r, c) */
                for (int f = g->row_ptr[r]; f < g->row_ptr[r + 1]; f++)
                    if (g->col[f] == c) { g->vn_edge[k] = f; break; }
                g->vn_row[k] = r;
                k++;
            }
    }
    g->vn_ptr[n] = k;
    return 0;
}

static void graph_free(graph_t *g) {
    free(g->row_ptr); free(g->col); free(g->vn_ptr); free(g->vn_edge); free(g->vn_row);
}

/* H e = s ?  (e, s as 0/1 bytes).  Returns 1 when every check is satisfied. */
static int syndrome_matches(const graph_t *g, const uint8_t *e, const uint8_t *s) {
    for (int r = 0; r < g->m; r++) {
        int par = 0;
        for (int f = g->row_ptr[r]; f < g->row_ptr[r + 1]; f++) par ^= e[g->col[f]];
        if (par != (s[r] & 1)) return 0;
    }
    return 1;
}

int orc_syndrome(int m, int n, const uint8_t *H, int nshots, const uint8_t *e, uint8_t *s) {
    for (int b = 0; b < nshots; b++)
        for (int r = 0; r < m; r++) {
            int par = 0;
            for (int c = 0; c < n; c++) par ^= (H[(long)r * n + c] != 0) & (e[(long)b * n + c] & 1);
            s[(long)b * m + r] = (uint8_t)par;
        }
    return 0;
}

static inline int sg_f(float x) { return x < 0.0f ? -1 : 1; }
static inline int sg_d(double x) { return x < 0.0 ? -1 : 1; }
static inline int sg_i(int x) { return x < 0 ? -1 : 1; }

/* ---------------------------------------------------------------------- */
/* Check-node rule, Algorithm 1: for each edge (m, n) of check m,          */
/*   r_{m,n} = (-1)^{s_m} prod_{j != n} sg(q_{m,j}) * scale * min_{j != n}|q_{m,j}|. */
/* scale is alpha, or the per-edge neural weight.                          */
/* ---------------------------------------------------------------------- */
static void cn_f32(const graph_t *g, int r, int s_bit, const float *q, float *rout,
                   float alpha, const float *w /* nullable, indexed by edge */) {
    int lo = g->row_ptr[r], hi = g->row_ptr[r + 1];
    for (int i = lo; i < hi; i++) {
        float mag = INFINITY;
        int sgn = s_bit ? -1 : 1;
        for (int j = lo; j < hi; j++) {
            if (j == i) continue;
            float a = fabsf(q[j]);
            if (a < mag) mag = a;
            sgn *= sg_f(q[j]);
        }
        float scale = w ? w[i] : alpha;
        float v = scale * mag;
        rout[i] = sgn < 0 ? -v : v;
    }
}

static void cn_f64(const graph_t *g, int r, int s_bit, const double *q, double *rout,
                   const double *w) {
    int lo = g->row_ptr[r], hi = g->row_ptr[r + 1];
    for (int i = lo; i < hi; i++) {
        double mag = INFINITY;
        int sgn = s_bit ? -1 : 1;
        for (int j = lo; j < hi; j++) {
            if (j == i) continue;
            double a = fabs(q[j]);
            if (a < mag) mag = a;
            sgn *= sg_d(q[j]);
        }
        double v = w[i] * mag;
        rout[i] = sgn < 0 ? -v : v;
    }
}

/* Fixed-point check rule (int8 and int16 messages): magnitudes are |q| in  */
/* [0, qmax]; alpha = num / 2^sh is applied to the magnitude and rounded    */
/* down, before the sign.                                                   */
static void cn_fx(const graph_t *g, int r, int s_bit, const int *q, int *rout, int num, int sh) {
    int lo = g->row_ptr[r], hi = g->row_ptr[r + 1];
    for (int i = lo; i < hi; i++) {
        int mag = 1 << 30;
        int sgn = s_bit ? -1 : 1;
        for (int j = lo; j < hi; j++) {
            if (j == i) continue;
            int a = q[j] < 0 ? -q[j] : q[j];
            if (a < mag) mag = a;
            sgn *= sg_i(q[j]);
        }
        int v = (num * mag) >> sh;
        rout[i] = sgn * v;
    }
}

static inline int clampq(int x, int qmax) { return x > qmax ? qmax : (x < -qmax ? -qmax : x); }

/* Fixed-point formats.  Messages saturate symmetrically to [-qmax, qmax];  */
/* priors are signed fixed point with `frac` fraction bits, held in        */
/* `bits`-bit integers; the reported posterior is Q / 2^frac.              */
/*   int8:  qmax = 127,   Q4 priors (frac = 4);                            */
/*   int16: qmax = 32767, Q8 priors (frac = 8).                            */
typedef struct { int bits, qmax, frac; } fxfmt_t;
static const fxfmt_t FX_I8 = {8, 127, 4};
static const fxfmt_t FX_I16 = {16, 32767, 8};

static inline int prior_at(const void *p, fxfmt_t f, long i) {
    return f.bits == 8 ? (int)((const int8_t *)p)[i] : (int)((const int16_t *)p)[i];
}

/* ---------------------------------------------------------------------- */
/* Flooding schedule, FP32 (Algorithm 1).  Optional per-iteration weights   */
/* w[k-1][e] replace alpha (neural min-sum) in iterations k <= wT; later    */
/* iterations use alpha (plain min-sum continuing from the neural state,    */
/* the continuation fallback).  Optional outputs: final                     */
/* posterior Q [B][n], every iteration's posterior Q_all [iters][B][n], and */
/* the inputs of every check-node pass q_traj [iters][B][nnz] (q^{(k-1)}).  */
/* ---------------------------------------------------------------------- */
int orc_flood_f32(int m, int n, const uint8_t *H, int nshots,
                  const uint8_t *syn, const float *prior, float alpha,
                  const float *w, int wT, int max_iters, int early_stop,
                  uint8_t *e_out, uint8_t *conv, int32_t *iters,
                  float *Q_out, float *Q_all, float *q_traj, int nthreads) {
    graph_t g;
    if (graph_build(&g, m, n, H)) return -1;
    int nnz = g.nnz;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int b = 0; b < nshots; b++) {
        const uint8_t *s = syn + (long)b * m;
        const float *gam = prior + (long)b * n;
        uint8_t *e = e_out + (long)b * n;
        float *q = malloc(sizeof(float) * (nnz + 1));
        float *rr = malloc(sizeof(float) * (nnz + 1));
        float *Q = malloc(sizeof(float) * (n + 1));
        /* initialisation: q^(0)_{m,n} = gamma_n */
        for (int c = 0; c < n; c++)
            for (int k = g.vn_ptr[c]; k < g.vn_ptr[c + 1]; k++) q[g.vn_edge[k]] = gam[c];
        int done = 0, k;
        for (k = 1; k <= max_iters; k++) {
            if (q_traj) memcpy(q_traj + ((long)(k - 1) * nshots + b) * nnz, q, sizeof(float) * nnz);
            const float *wk = (w && k <= wT) ? w + (long)(k - 1) * nnz : NULL;
            for (int r = 0; r < m; r++) cn_f32(&g, r, s[r] & 1, q, rr, alpha, wk);
            /* variable nodes: excluded sums in increasing check order */
            for (int c = 0; c < n; c++) {
                int lo = g.vn_ptr[c], hi = g.vn_ptr[c + 1];
                for (int i = lo; i < hi; i++) {
                    float acc = gam[c];
                    for (int j = lo; j < hi; j++)
                        if (j != i) acc = acc + rr[g.vn_edge[j]];
                    q[g.vn_edge[i]] = acc;
                }
                float acc = gam[c];
                for (int j = lo; j < hi; j++) acc = acc + rr[g.vn_edge[j]];
                Q[c] = acc;
                e[c] = Q[c] < 0.0f ? 1 : 0;
            }
            if (Q_all) memcpy(Q_all + ((long)(k - 1) * nshots + b) * n, Q, sizeof(float) * n);
            if (early_stop && syndrome_matches(&g, e, s)) { done = 1; break; }
        }
        if (done) {
            conv[b] = 1;
            iters[b] = k;
        } else {
            conv[b] = (uint8_t)syndrome_matches(&g, e, s);
            iters[b] = max_iters;
        }
        if (Q_out) memcpy(Q_out + (long)b * n, Q, sizeof(float) * n);
        free(q); free(rr); free(Q);
    }
    graph_free(&g);
    return 0;
}

/* Flooding, fixed-point messages.  q and r live in [-qmax, qmax]; sums    */
/* are exact int32 and saturate only where a message is formed.            */
static int flood_fx(int m, int n, const uint8_t *H, int nshots,
                    const uint8_t *syn, const void *prior, fxfmt_t f, int alpha_num, int alpha_shift,
                    int max_iters, int early_stop,
                    uint8_t *e_out, uint8_t *conv, int32_t *iters, float *Q_out, int nthreads) {
    graph_t g;
    if (graph_build(&g, m, n, H)) return -1;
    int nnz = g.nnz;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int b = 0; b < nshots; b++) {
        const uint8_t *s = syn + (long)b * m;
        uint8_t *e = e_out + (long)b * n;
        int *q = malloc(sizeof(int) * (nnz + 1));
        int *rr = malloc(sizeof(int) * (nnz + 1));
        int *Q = malloc(sizeof(int) * (n + 1));
        int *gam = malloc(sizeof(int) * (n + 1));
        for (int c = 0; c < n; c++) gam[c] = prior_at(prior, f, (long)b * n + c);
        for (int c = 0; c < n; c++)
            for (int k = g.vn_ptr[c]; k < g.vn_ptr[c + 1]; k++) q[g.vn_edge[k]] = gam[c];
        int done = 0, k;
        for (k = 1; k <= max_iters; k++) {
            for (int r = 0; r < m; r++) cn_fx(&g, r, s[r] & 1, q, rr, alpha_num, alpha_shift);
            for (int c = 0; c < n; c++) {
                int lo = g.vn_ptr[c], hi = g.vn_ptr[c + 1];
                for (int i = lo; i < hi; i++) {
                    int acc = gam[c];
                    for (int j = lo; j < hi; j++)
                        if (j != i) acc += rr[g.vn_edge[j]];
                    q[g.vn_edge[i]] = clampq(acc, f.qmax);
                }
                int acc = gam[c];
                for (int j = lo; j < hi; j++) acc += rr[g.vn_edge[j]];
                Q[c] = acc;
                e[c] = Q[c] < 0 ? 1 : 0;
            }
            if (early_stop && syndrome_matches(&g, e, s)) { done = 1; break; }
        }
        if (done) { conv[b] = 1; iters[b] = k; }
        else { conv[b] = (uint8_t)syndrome_matches(&g, e, s); iters[b] = max_iters; }
        if (Q_out)
            for (int c = 0; c < n; c++) Q_out[(long)b * n + c] = (float)Q[c] / (float)(1 << f.frac);
        free(q); free(rr); free(Q); free(gam);
    }
    graph_free(&g);
    return 0;
}

int orc_flood_i8(int m, int n, const uint8_t *H, int nshots,
                 const uint8_t *syn, const int8_t *prior_q4, int alpha_num, int alpha_shift,
                 int max_iters, int early_stop,
                 uint8_t *e_out, uint8_t *conv, int32_t *iters, float *Q_out, int nthreads) {
    return flood_fx(m, n, H, nshots, syn, prior_q4, FX_I8, alpha_num, alpha_shift, max_iters,
                    early_stop, e_out, conv, iters, Q_out, nthreads);
}

int orc_flood_i16(int m, int n, const uint8_t *H, int nshots,
                  const uint8_t *syn, const int16_t *prior_q8, int alpha_num, int alpha_shift,
                  int max_iters, int early_stop,
                  uint8_t *e_out, uint8_t *conv, int32_t *iters, float *Q_out, int nthreads) {
    return flood_fx(m, n, H, nshots, syn, prior_q8, FX_I16, alpha_num, alpha_shift, max_iters,
                    early_stop, e_out, conv, iters, Q_out, nthreads);
}

/* ---------------------------------------------------------------------- */
/* Row-layered schedule.  Checks are grouped into layers given by           */
/* layer_ptr[0..nlayers] (checks layer_ptr[l] .. layer_ptr[l+1]-1); layers  */
/* run in increasing order and checks within a layer in increasing index.   */
/* Per check: q_e = Q_n - r_e, new r from those q as in the check rule,     */
/* then Q_n = q_e + r_new_e.  One sweep over all layers is one iteration,   */
/* followed by the decision and the syndrome test.  Starting state: Q =     */
/* gamma, r = 0.  Fixed point: the check rule reads the saturated message  */
/* q_e = clamp(Q_n - r_e, -qmax, qmax), while the posterior is updated      */
/* exactly, Q_n = (Q_n - r_e) + r_new_e, so Q_n = gamma_n + sum of the      */
/* current r of its checks at all times (|Q_n| <= qmax + d_v * alpha qmax). */
/* ---------------------------------------------------------------------- */
int orc_layered_f32(int m, int n, const uint8_t *H, int nshots,
                    const uint8_t *syn, const float *prior, float alpha,
                    int nlayers, const int32_t *layer_ptr, int max_iters, int early_stop,
                    uint8_t *e_out, uint8_t *conv, int32_t *iters, float *Q_out, int nthreads) {
    graph_t g;
    if (graph_build(&g, m, n, H)) return -1;
    int nnz = g.nnz;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int b = 0; b < nshots; b++) {
        const uint8_t *s = syn + (long)b * m;
        const float *gam = prior + (long)b * n;
        uint8_t *e = e_out + (long)b * n;
        float *rr = calloc((size_t)nnz + 1, sizeof(float));
        float *qloc = malloc(sizeof(float) * (nnz + 1));
        float *rnew = malloc(sizeof(float) * (nnz + 1));
        float *Q = malloc(sizeof(float) * (n + 1));
        for (int c = 0; c < n; c++) Q[c] = gam[c];
        int done = 0, k;
        for (k = 1; k <= max_iters; k++) {
            for (int l = 0; l < nlayers; l++)
                for (int r = layer_ptr[l]; r < layer_ptr[l + 1]; r++) {
                    int lo = g.row_ptr[r], hi = g.row_ptr[r + 1];
                    for (int f = lo; f < hi; f++) qloc[f] = Q[g.col[f]] - rr[f];
                    cn_f32(&g, r, s[r] & 1, qloc, rnew, alpha, NULL);
                    for (int f = lo; f < hi; f++) {
                        Q[g.col[f]] = qloc[f] + rnew[f];
                        rr[f] = rnew[f];
                    }
                }
            for (int c = 0; c < n; c++) e[c] = Q[c] < 0.0f ? 1 : 0;
            if (early_stop && syndrome_matches(&g, e, s)) { done = 1; break; }
        }
        if (done) { conv[b] = 1; iters[b] = k; }
        else { conv[b] = (uint8_t)syndrome_matches(&g, e, s); iters[b] = max_iters; }
        if (Q_out) memcpy(Q_out + (long)b * n, Q, sizeof(float) * n);
        free(rr); free(qloc); free(rnew); free(Q);
    }
    graph_free(&g);
    return 0;
}

static int layered_fx(int m, int n, const uint8_t *H, int nshots,
                      const uint8_t *syn, const void *prior, fxfmt_t f, int alpha_num, int alpha_shift,
                      int nlayers, const int32_t *layer_ptr, int max_iters, int early_stop,
                      uint8_t *e_out, uint8_t *conv, int32_t *iters, float *Q_out, int nthreads) {
    graph_t g;
    if (graph_build(&g, m, n, H)) return -1;
    int nnz = g.nnz;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int b = 0; b < nshots; b++) {
        const uint8_t *s = syn + (long)b * m;
        uint8_t *e = e_out + (long)b * n;
        int *rr = calloc((size_t)nnz + 1, sizeof(int));
        int *qloc = malloc(sizeof(int) * (nnz + 1));
        int *rnew = malloc(sizeof(int) * (nnz + 1));
        int *Q = malloc(sizeof(int) * (n + 1));
        for (int c = 0; c < n; c++) Q[c] = prior_at(prior, f, (long)b * n + c);
        int done = 0, k;
        for (k = 1; k <= max_iters; k++) {
            for (int l = 0; l < nlayers; l++)
                for (int r = layer_ptr[l]; r < layer_ptr[l + 1]; r++) {
                    int lo = g.row_ptr[r], hi = g.row_ptr[r + 1];
                    for (int x = lo; x < hi; x++) qloc[x] = clampq(Q[g.col[x]] - rr[x], f.qmax);
                    cn_fx(&g, r, s[r] & 1, qloc, rnew, alpha_num, alpha_shift);
                    for (int x = lo; x < hi; x++) {
                        Q[g.col[x]] = (Q[g.col[x]] - rr[x]) + rnew[x];
                        rr[x] = rnew[x];
                    }
                }
            for (int c = 0; c < n; c++) e[c] = Q[c] < 0 ? 1 : 0;
            if (early_stop && syndrome_matches(&g, e, s)) { done = 1; break; }
        }
        if (done) { conv[b] = 1; iters[b] = k; }
        else { conv[b] = (uint8_t)syndrome_matches(&g, e, s); iters[b] = max_iters; }
        if (Q_out)
            for (int c = 0; c < n; c++) Q_out[(long)b * n + c] = (float)Q[c] / (float)(1 << f.frac);
        free(rr); free(qloc); free(rnew); free(Q);
    }
    graph_free(&g);
    return 0;
}

int orc_layered_i8(int m, int n, const uint8_t *H, int nshots,
                   const uint8_t *syn, const int8_t *prior_q4, int alpha_num, int alpha_shift,
                   int nlayers, const int32_t *layer_ptr, int max_iters, int early_stop,
                   uint8_t *e_out, uint8_t *conv, int32_t *iters, float *Q_out, int nthreads) {
    return layered_fx(m, n, H, nshots, syn, prior_q4, FX_I8, alpha_num, alpha_shift, nlayers, layer_ptr,
                      max_iters, early_stop, e_out, conv, iters, Q_out, nthreads);
}

int orc_layered_i16(int m, int n, const uint8_t *H, int nshots,
                    const uint8_t *syn, const int16_t *prior_q8, int alpha_num, int alpha_shift,
                    int nlayers, const int32_t *layer_ptr, int max_iters, int early_stop,
                    uint8_t *e_out, uint8_t *conv, int32_t *iters, float *Q_out, int nthreads) {
    return layered_fx(m, n, H, nshots, syn, prior_q8, FX_I16, alpha_num, alpha_shift, nlayers, layer_ptr,
                      max_iters, early_stop, e_out, conv, iters, Q_out, nthreads);
}

/* ---------------------------------------------------------------------- */
/* Neural min-sum in double precision: flooding with weights w[k-1][e] in   */
/* place of alpha, T iterations, no early stop.  Emits every iteration's    */
/* posterior Q_all [T][B][n] and the check-node inputs q_traj [T][B][nnz].  */
/* Used for finite-difference checks of the adjoint below.                  */
/* ---------------------------------------------------------------------- */
int orc_nms_forward_f64(int m, int n, const uint8_t *H, int nshots,
                        const uint8_t *syn, const double *prior, const double *w, int T,
                        double *Q_all, double *q_traj, int nthreads) {
    graph_t g;
    if (graph_build(&g, m, n, H)) return -1;
    int nnz = g.nnz;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int b = 0; b < nshots; b++) {
        const uint8_t *s = syn + (long)b * m;
        const double *gam = prior + (long)b * n;
        double *q = malloc(sizeof(double) * (nnz + 1));
        double *rr = malloc(sizeof(double) * (nnz + 1));
        for (int c = 0; c < n; c++)
            for (int k = g.vn_ptr[c]; k < g.vn_ptr[c + 1]; k++) q[g.vn_edge[k]] = gam[c];
        for (int k = 1; k <= T; k++) {
            if (q_traj) memcpy(q_traj + ((long)(k - 1) * nshots + b) * nnz, q, sizeof(double) * nnz);
            for (int r = 0; r < m; r++) cn_f64(&g, r, s[r] & 1, q, rr, w + (long)(k - 1) * nnz);
            double *Qk = Q_all + ((long)(k - 1) * nshots + b) * n;
            for (int c = 0; c < n; c++) {
                int lo = g.vn_ptr[c], hi = g.vn_ptr[c + 1];
                for (int i = lo; i < hi; i++) {
                    double acc = gam[c];
                    for (int j = lo; j < hi; j++)
                        if (j != i) acc = acc + rr[g.vn_edge[j]];
                    q[g.vn_edge[i]] = acc;
                }
                double acc = gam[c];
                for (int j = lo; j < hi; j++) acc = acc + rr[g.vn_edge[j]];
                Qk[c] = acc;
            }
        }
        free(q); free(rr);
    }
    graph_free(&g);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Adjoint of neural min-sum (reverse-mode derivative of the forward map    */
/* above, written out by hand).  Inputs: the check-node inputs q^{(k-1)}    */
/* of every iteration (q_traj [T][B][nnz], from either forward), weights,   */
/* syndrome, and G[k-1][b][n] = dL/dQ^{(k)}_n.  Sweeping k = T .. 1:        */
/*   g_r^{(k)}_{m,n}  = G^{(k)}_n + sum_{i in S_c(n), i != m} g_q^{(k)}_{i,n} */
/*   dL/dw^{(k)}_e   += g_r^{(k)}_e * sgn_e * mag_e                          */
/*   g_q^{(k-1)}_{m,a} += g_r^{(k)}_{m,n} * w^{(k)}_e * sgn_e * sg(q_{m,a})   */
/* where a is the argmin of |q^{(k-1)}| over S_v(m) \ n (ties: lowest edge  */
/* index) and sgn_e the sign of r_e.  Signs carry no gradient.  g_q^{(T)}   */
/* is zero.  grad_w [T][nnz] receives the sum over shots; grad_abs the sum  */
/* of absolute per-shot contributions (a scale for rounding tolerances).    */
/* ---------------------------------------------------------------------- */
int orc_nms_adjoint_f64(int m, int n, const uint8_t *H, int nshots,
                        const uint8_t *syn, const double *w, int T,
                        const double *q_traj, const double *G,
                        double *grad_w, double *grad_abs) {
    graph_t g;
    if (graph_build(&g, m, n, H)) return -1;
    int nnz = g.nnz;
    memset(grad_w, 0, sizeof(double) * (size_t)T * nnz);
    if (grad_abs) memset(grad_abs, 0, sizeof(double) * (size_t)T * nnz);
    double *gq = malloc(sizeof(double) * (nnz + 1));
    double *gq_prev = malloc(sizeof(double) * (nnz + 1));
    double *gr = malloc(sizeof(double) * (nnz + 1));
    for (int b = 0; b < nshots; b++) {
        const uint8_t *s = syn + (long)b * m;
        for (int f = 0; f < nnz; f++) gq[f] = 0.0;
        for (int k = T; k >= 1; k--) {
            const double *q = q_traj + ((long)(k - 1) * nshots + b) * nnz;
            const double *wk = w + (long)(k - 1) * nnz;
            const double *Gk = G + ((long)(k - 1) * nshots + b) * n;
            /* g_r from the variable-node side */
            for (int c = 0; c < n; c++) {
                int lo = g.vn_ptr[c], hi = g.vn_ptr[c + 1];
                for (int i = lo; i < hi; i++) {
                    double acc = Gk[c];
                    for (int j = lo; j < hi; j++)
                        if (j != i) acc += gq[g.vn_edge[j]];
                    gr[g.vn_edge[i]] = acc;
                }
            }
            for (int f = 0; f < nnz; f++) gq_prev[f] = 0.0;
            /* through the check-node rule */
            for (int r = 0; r < m; r++) {
                int lo = g.row_ptr[r], hi = g.row_ptr[r + 1];
                for (int i = lo; i < hi; i++) {
                    double mag = INFINITY;
                    int arg = -1;
                    int sgn = (s[r] & 1) ? -1 : 1;
                    for (int j = lo; j < hi; j++) {
                        if (j == i) continue;
                        double a = fabs(q[j]);
                        if (a < mag) { mag = a; arg = j; }
                        sgn *= sg_d(q[j]);
                    }
                    double contrib = gr[i] * (double)sgn * mag;
                    grad_w[(long)(k - 1) * nnz + i] += contrib;
                    if (grad_abs) grad_abs[(long)(k - 1) * nnz + i] += fabs(contrib);
                    gq_prev[arg] += gr[i] * wk[i] * (double)sgn * (double)sg_d(q[arg]);
                }
            }
            double *t = gq; gq = gq_prev; gq_prev = t;
        }
    }
    free(gq); free(gq_prev); free(gr);
    graph_free(&g);
    return 0;
}

int orc_edge_count(int m, int n, const uint8_t *H) {
    int nnz = 0;
    for (long i = 0; i < (long)m * n; i++) nnz += H[i] != 0;
    return nnz;
}
