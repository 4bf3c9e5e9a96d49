/*
 * Plain CPU oracle for Spiking Neural Dedispersion (SND).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link or call
 * this file; only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It is written from the paper (Methods: "The neuromorphic dedispersion
 * neuron", "Input encoding", "Incoherent dedispersion", "The Spiking Neural
 * Dedispersion algorithm", "Matched filtering", "Candidate detection") and shares no
 * code, header or table with the GPU library.
 *
 * Arithmetic: every value is held in IEEE double.  Integer modes therefore compute
 * exact integer sums (all sums here stay far below 2^53).  Compile with
 * -ffp-contract=off so that no multiply-add is fused.
 *
 * Readings of points the paper leaves open:
 *  - delays are rounded half-to-even from one fixed FP64 expression;
 *  - the output time origin is the arrival time at the reference frequency, i.e. the
 *    "t + delta" form y_d(t) = sum_c x_c(t + delta_c(d));
 *  - the reference channel of a tree node is its highest-frequency channel and node
 *    shifts are differences of the globally rounded channel delays;
 *  - the binary quorum is "count >= K" with K_L at leaves and K_I at every higher
 *    node including the root; graded clipping applies at every node;
 *  - a binary-mode input sample counts as a spike when it is non-zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_KDM 4.148808e6 /* MHz^2 ms per pc cm^-3 */
#define ORC_MAXLEV 48

enum { ORC_BINARY = 0, ORC_GRADED = 1, ORC_FLOAT = 2 };
enum { ORC_IN_U8 = 0, ORC_IN_F32 = 1, ORC_IN_F64 = 2 };

typedef struct {
    int32_t mode;       /* ORC_BINARY / ORC_GRADED / ORC_FLOAT */
    int32_t cluster;    /* C: channels per leaf cluster */
    int32_t branching;  /* B: children per internal node */
    int32_t k_leaf;     /* binary quorum at leaves */
    int32_t k_int;      /* binary quorum at every higher node */
    int32_t cap;        /* graded clip value N */
    int32_t root_norm;  /* float: divide the root by sqrt(nchan) */
} orc_params;

/* ------------------------------------------------------------------------------------
 * Dispersive delays (Methods, "Incoherent dedispersion"): the cold-plasma delay between
 * frequencies f and f_ref is K_DM * DM * (f^-2 - f_ref^-2) ms; the integer per-channel
 * delay is that value divided by the sampling interval and rounded to nearest.
 * out[k * nchan + c] = delta_c(dm[k]).  fref <= 0 selects max(freq).
 * Returns 0, or -1 when fref is below the highest channel frequency.
 * ---------------------------------------------------------------------------------- */
int orc_delays(int32_t nchan, const double *freq, double tsamp_s, double fref, int32_t ndm,
               const double *dm, int32_t *out)
{
    double fmax = freq[0];
    for (int32_t c = 1; c < nchan; ++c)
        if (freq[c] > fmax) fmax = freq[c];
    double fr = fref > 0.0 ? fref : fmax;
    if (fr < fmax) return -1;
    double tms = tsamp_s * 1e3;
    for (int32_t k = 0; k < ndm; ++k) {
        for (int32_t c = 0; c < nchan; ++c) {
            double x = ORC_KDM * dm[k];
            x = x * (1.0 / (freq[c] * freq[c]) - 1.0 / (fr * fr));
            x = x / tms;
            out[(int64_t)k * nchan + c] = (int32_t)nearbyint(x);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Tree shape (Methods, SND "Leaf clusters" and "Tree levels"): contiguous clusters of C
 * channels (the last one may be smaller) form level 0; each higher level groups B
 * consecutive nodes of the level below (the last group may be smaller) until a single
 * root remains.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int32_t nlev;
    int32_t nnodes[ORC_MAXLEV];
    int32_t *chlo[ORC_MAXLEV], *chhi[ORC_MAXLEV]; /* channel range of each node */
    int32_t *kidlo[ORC_MAXLEV], *kidhi[ORC_MAXLEV]; /* child-node range (levels >= 1) */
    int32_t *ref[ORC_MAXLEV]; /* reference channel: highest frequency, lowest index on ties */
} orc_tree;

static void tree_free(orc_tree *t)
{
    for (int l = 0; l < t->nlev; ++l) {
        free(t->chlo[l]); free(t->chhi[l]); free(t->kidlo[l]); free(t->kidhi[l]); free(t->ref[l]);
    }
    t->nlev = 0;
}

static int tree_build(orc_tree *t, int32_t nchan, const double *freq, int32_t C, int32_t B)
{
    memset(t, 0, sizeof(*t));
    if (nchan < 1 || C < 1 || B < 2) return -1;
    int32_t n = (nchan + C - 1) / C;
    int l = 0;
    for (;;) {
        if (l >= ORC_MAXLEV) { tree_free(t); return -1; }
        t->nnodes[l] = n;
        t->chlo[l] = malloc(sizeof(int32_t) * n); t->chhi[l] = malloc(sizeof(int32_t) * n);
        t->kidlo[l] = malloc(sizeof(int32_t) * n); t->kidhi[l] = malloc(sizeof(int32_t) * n);
        t->ref[l] = malloc(sizeof(int32_t) * n);
        for (int32_t i = 0; i < n; ++i) {
            if (l == 0) {
                t->kidlo[0][i] = t->kidhi[0][i] = 0;
                t->chlo[0][i] = i * C;
                t->chhi[0][i] = (i + 1) * C < nchan ? (i + 1) * C : nchan;
            } else {
                int32_t a = i * B, b = (i + 1) * B < t->nnodes[l - 1] ? (i + 1) * B : t->nnodes[l - 1];
                t->kidlo[l][i] = a; t->kidhi[l][i] = b;
                t->chlo[l][i] = t->chlo[l - 1][a];
                t->chhi[l][i] = t->chhi[l - 1][b - 1];
            }
            int32_t r = t->chlo[l][i];
            for (int32_t c = t->chlo[l][i] + 1; c < t->chhi[l][i]; ++c)
                if (freq[c] > freq[r]) r = c;
            t->ref[l][i] = r;
        }
        t->nlev = l + 1;
        if (n == 1) break;
        n = (n + B - 1) / B;
        ++l;
    }
    return 0;
}

/* Query the shape: nodes per level (leaf first); returns the number of levels. */
int orc_tree_shape(int32_t nchan, const double *freq, int32_t C, int32_t B, int32_t *nodes_out, int32_t maxlev)
{
    orc_tree t;
    if (tree_build(&t, nchan, freq, C, B)) return -1;
    int nl = t.nlev;
    for (int l = 0; l < nl && l < maxlev; ++l) nodes_out[l] = t.nnodes[l];
    tree_free(&t);
    return nl;
}

/* ------------------------------------------------------------------------------------
 * Node activation (Methods, "Tree activation modes"; cascade quorum in Results):
 *   binary: 1 when the count of active inputs meets or exceeds K (K_L at leaves, K_I
 *           above), else 0;
 *   graded: the integer sum clipped to [0, N];
 *   float : the sum itself.
 * ---------------------------------------------------------------------------------- */
static double phi(const orc_params *p, int leaf, double a)
{
    if (p->mode == ORC_BINARY) return a >= (double)(leaf ? p->k_leaf : p->k_int) ? 1.0 : 0.0;
    if (p->mode == ORC_GRADED) return a > (double)p->cap ? (double)p->cap : a;
    return a;
}

typedef struct {
    const void *x;
    int32_t xtype;
    int64_t nt;
    int32_t mode;
} orc_input;

/* Input sample of channel c at time t; binary mode counts any non-zero sample as one spike. */
static double xin(const orc_input *in, int32_t c, int64_t t)
{
    int64_t i = (int64_t)c * in->nt + t;
    double v;
    if (in->xtype == ORC_IN_U8) v = (double)((const uint8_t *)in->x)[i];
    else if (in->xtype == ORC_IN_F32) v = (double)((const float *)in->x)[i];
    else v = ((const double *)in->x)[i];
    if (in->mode == ORC_BINARY) v = v != 0.0 ? 1.0 : 0.0;
    return v;
}

static int64_t max_delay(const int32_t *delays, int32_t ndm, int32_t nchan)
{
    int64_t m = 0;
    for (int64_t i = 0; i < (int64_t)ndm * nchan; ++i)
        if (delays[i] > m) m = delays[i];
    return m;
}

/* ------------------------------------------------------------------------------------
 * Reference recursion, no sharing between DMs (the definition the dedup tree must equal).
 * A node's value at its own reference time t sums its inputs shifted by their delay
 * relative to the node's reference channel (Methods, "The neuromorphic dedispersion
 * neuron": v(t) = sum_i w_i s_i(t - delta_i) with unit weights, written here in the
 * arrival-at-reference form), then applies the node activation.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    const orc_tree *tr;
    const orc_params *p;
    const orc_input *in;
    const int32_t *dk; /* delays of one DM, [nchan] */
} orc_ctx;

static double eval_node(const orc_ctx *cx, int lev, int32_t node, int64_t t)
{
    const orc_tree *tr = cx->tr;
    int32_t r = tr->ref[lev][node];
    double a = 0.0;
    if (lev == 0) {
        for (int32_t c = tr->chlo[0][node]; c < tr->chhi[0][node]; ++c)
            a += xin(cx->in, c, t + cx->dk[c] - cx->dk[r]);
    } else {
        for (int32_t j = tr->kidlo[lev][node]; j < tr->kidhi[lev][node]; ++j)
            a += eval_node(cx, lev - 1, j, t + cx->dk[tr->ref[lev - 1][j]] - cx->dk[r]);
    }
    return phi(cx->p, lev == 0, a);
}

static double root_value(const orc_ctx *cx, int64_t t, int32_t nchan)
{
    int top = cx->tr->nlev - 1;
    double v = eval_node(cx, top, 0, t + cx->dk[cx->tr->ref[top][0]]);
    if (cx->p->mode == ORC_FLOAT && cx->p->root_norm) v = v / sqrt((double)nchan);
    return v;
}

/* Sampled outputs y[k_i][t_i] of the reference recursion; returns 0 or -1 on a bad argument. */
int orc_snd_points(const orc_params *p, int32_t nchan, const double *freq, int64_t nt, const void *x,
                   int32_t xtype, int32_t ndm, const int32_t *delays, int64_t npts, const int32_t *ks,
                   const int64_t *ts, double *out)
{
    orc_tree tr;
    if (tree_build(&tr, nchan, freq, p->cluster, p->branching)) return -1;
    int64_t nout = nt - max_delay(delays, ndm, nchan);
    orc_input in = {x, xtype, nt, p->mode};
    int rc = 0;
    for (int64_t i = 0; i < npts; ++i) {
        if (ks[i] < 0 || ks[i] >= ndm || ts[i] < 0 || ts[i] >= nout) { rc = -1; break; }
        orc_ctx cx = {&tr, p, &in, delays + (int64_t)ks[i] * nchan};
        out[i] = root_value(&cx, ts[i], nchan);
    }
    tree_free(&tr);
    return rc;
}

/* Whole DM-time plane by the reference recursion: y[k][t], t in [0, nt - max delay). */
int orc_snd_recursive(const orc_params *p, int32_t nchan, const double *freq, int64_t nt, const void *x,
                      int32_t xtype, int32_t ndm, const int32_t *delays, double *y)
{
    orc_tree tr;
    if (tree_build(&tr, nchan, freq, p->cluster, p->branching)) return -1;
    int64_t nout = nt - max_delay(delays, ndm, nchan);
    if (nout <= 0) { tree_free(&tr); return -1; }
    orc_input in = {x, xtype, nt, p->mode};
    for (int32_t k = 0; k < ndm; ++k) {
        orc_ctx cx = {&tr, p, &in, delays + (int64_t)k * nchan};
        for (int64_t t = 0; t < nout; ++t) y[(int64_t)k * nout + t] = root_value(&cx, t, nchan);
    }
    tree_free(&tr);
    return 0;
}

/* Direct (brute-force) incoherent dedispersion: y[k][t] = sum_c x_c(t + delta_c(d_k)),
 * no activation (Methods, "The neuromorphic dedispersion neuron" and "Incoherent
 * dedispersion"); binary-mode inputs count non-zero samples as one. */
int orc_bruteforce(int32_t mode, int32_t nchan, int64_t nt, const void *x, int32_t xtype, int32_t ndm,
                   const int32_t *delays, double *y)
{
    int64_t nout = nt - max_delay(delays, ndm, nchan);
    if (nout <= 0) return -1;
    orc_input in = {x, xtype, nt, mode};
    for (int32_t k = 0; k < ndm; ++k) {
        const int32_t *dk = delays + (int64_t)k * nchan;
        for (int64_t t = 0; t < nout; ++t) {
            double a = 0.0;
            for (int32_t c = 0; c < nchan; ++c) a += xin(&in, c, t + dk[c]);
            y[(int64_t)k * nout + t] = a;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * The SND plan proper (Methods, SND): at every node the DMs are grouped by their delay
 * pattern -- at a leaf the tuple of channel delays relative to the node's reference
 * channel, above it the tuple of (child neuron, child shift) -- and each distinct
 * pattern is one neuron, evaluated once and shared by all DMs that have it.
 * ---------------------------------------------------------------------------------- */
static int g_keylen;
static int cmp_keyrec(const void *a, const void *b)
{
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    for (int i = 0; i < g_keylen; ++i) {
        if (x[i] < y[i]) return -1;
        if (x[i] > y[i]) return 1;
    }
    /* equal keys: order by the DM index stored after the key */
    return x[g_keylen] < y[g_keylen] ? -1 : x[g_keylen] > y[g_keylen];
}

typedef struct {
    int32_t nneu;     /* neurons at this node */
    int32_t *nid;     /* [ndm]: neuron serving each DM */
    int32_t *krep;    /* [nneu]: one DM served by each neuron */
    int64_t *lo, *hi; /* [nneu]: range of the node reference delay over the DMs served */
    double **val;     /* [nneu]: value at reference times lo .. hi + nout - 1 */
} orc_node;

static void node_free(orc_node *n)
{
    if (n->val) for (int32_t i = 0; i < n->nneu; ++i) free(n->val[i]);
    free(n->val); free(n->nid); free(n->krep); free(n->lo); free(n->hi);
    memset(n, 0, sizeof(*n));
}

/* counts[2*l] = neurons at level l, counts[2*l+1] = synapses (inputs) at level l. */
int orc_snd_dedup(const orc_params *p, int32_t nchan, const double *freq, int64_t nt, const void *x,
                  int32_t xtype, int32_t ndm, const int32_t *delays, double *y, int64_t *counts,
                  int32_t maxlev)
{
    orc_tree tr;
    if (tree_build(&tr, nchan, freq, p->cluster, p->branching)) return -1;
    int64_t nout = nt - max_delay(delays, ndm, nchan);
    if (nout <= 0 || ndm < 1) { tree_free(&tr); return -1; }
    orc_input in = {x, xtype, nt, p->mode};
    orc_node *prev = NULL;
    int32_t nprev = 0;
    for (int lev = 0; lev < tr.nlev; ++lev) {
        int32_t nn = tr.nnodes[lev];
        orc_node *cur = calloc((size_t)nn, sizeof(orc_node));
        int64_t nneu_lev = 0, nsyn_lev = 0;
        for (int32_t node = 0; node < nn; ++node) {
            orc_node *nd = &cur[node];
            int32_t r = tr.ref[lev][node];
            int32_t fan = lev == 0 ? tr.chhi[0][node] - tr.chlo[0][node] : tr.kidhi[lev][node] - tr.kidlo[lev][node];
            int keylen = lev == 0 ? fan : 2 * fan;
            int64_t *rec = malloc(sizeof(int64_t) * (size_t)(keylen + 1) * (size_t)ndm);
            for (int32_t k = 0; k < ndm; ++k) {
                const int32_t *dk = delays + (int64_t)k * nchan;
                int64_t *kr = rec + (int64_t)k * (keylen + 1);
                if (lev == 0) {
                    for (int32_t i = 0; i < fan; ++i) kr[i] = dk[tr.chlo[0][node] + i] - dk[r];
                } else {
                    for (int32_t i = 0; i < fan; ++i) {
                        int32_t ch = tr.kidlo[lev][node] + i;
                        kr[2 * i] = prev[ch].nid[k];
                        kr[2 * i + 1] = dk[tr.ref[lev - 1][ch]] - dk[r];
                    }
                }
                kr[keylen] = k;
            }
            g_keylen = keylen;
            qsort(rec, (size_t)ndm, sizeof(int64_t) * (size_t)(keylen + 1), cmp_keyrec);
            nd->nid = malloc(sizeof(int32_t) * (size_t)ndm);
            nd->krep = malloc(sizeof(int32_t) * (size_t)ndm);
            nd->lo = malloc(sizeof(int64_t) * (size_t)ndm);
            nd->hi = malloc(sizeof(int64_t) * (size_t)ndm);
            int32_t nu = 0;
            for (int32_t i = 0; i < ndm; ++i) {
                int64_t *kr = rec + (int64_t)i * (keylen + 1);
                int newkey = i == 0 || memcmp(kr, kr - (keylen + 1), sizeof(int64_t) * (size_t)keylen) != 0;
                int32_t k = (int32_t)kr[keylen];
                int64_t dr = delays[(int64_t)k * nchan + r];
                if (newkey) {
                    nd->krep[nu] = k;
                    nd->lo[nu] = dr;
                    nd->hi[nu] = dr;
                    ++nu;
                }
                nd->nid[k] = nu - 1;
                if (dr < nd->lo[nu - 1]) nd->lo[nu - 1] = dr;
                if (dr > nd->hi[nu - 1]) nd->hi[nu - 1] = dr;
            }
            free(rec);
            nd->nneu = nu;
            nneu_lev += nu;
            nsyn_lev += (int64_t)nu * fan;
            /* evaluate each neuron once over the reference times its DMs need */
            nd->val = calloc((size_t)nu, sizeof(double *));
            for (int32_t u = 0; u < nu; ++u) {
                const int32_t *dk = delays + (int64_t)nd->krep[u] * nchan;
                int64_t len = nd->hi[u] - nd->lo[u] + nout;
                double *v = malloc(sizeof(double) * (size_t)len);
                for (int64_t i = 0; i < len; ++i) {
                    int64_t t = nd->lo[u] + i;
                    double a = 0.0;
                    if (lev == 0) {
                        for (int32_t c = tr.chlo[0][node]; c < tr.chhi[0][node]; ++c)
                            a += xin(&in, c, t + dk[c] - dk[r]);
                    } else {
                        for (int32_t ch = tr.kidlo[lev][node]; ch < tr.kidhi[lev][node]; ++ch) {
                            const orc_node *cn = &prev[ch];
                            int32_t m = cn->nid[nd->krep[u]];
                            int64_t tc = t + dk[tr.ref[lev - 1][ch]] - dk[r];
                            a += cn->val[m][tc - cn->lo[m]];
                        }
                    }
                    v[i] = phi(p, lev == 0, a);
                }
                nd->val[u] = v;
            }
        }
        if (lev < maxlev) { counts[2 * lev] = nneu_lev; counts[2 * lev + 1] = nsyn_lev; }
        for (int32_t i = 0; i < nprev; ++i) node_free(&prev[i]);
        free(prev);
        prev = cur;
        nprev = nn;
    }
    /* root: one output row per DM */
    int top = tr.nlev - 1;
    orc_node *root = &prev[0];
    int32_t rr = tr.ref[top][0];
    for (int32_t k = 0; k < ndm; ++k) {
        int32_t m = root->nid[k];
        int64_t dr = delays[(int64_t)k * nchan + rr];
        for (int64_t t = 0; t < nout; ++t) {
            double v = root->val[m][t + dr - root->lo[m]];
            if (p->mode == ORC_FLOAT && p->root_norm) v = v / sqrt((double)nchan);
            y[(int64_t)k * nout + t] = v;
        }
    }
    for (int32_t i = 0; i < nprev; ++i) node_free(&prev[i]);
    free(prev);
    int nl = tr.nlev;
    tree_free(&tr);
    return nl;
}

/* ------------------------------------------------------------------------------------
 * Delta encoder (Methods, "Input encoding"): x = 1[z > theta].  With several thresholds
 * the level is the number of thresholds exceeded (the multi-level form of the same
 * comparison).  z and the thresholds are compared in single precision.
 * ---------------------------------------------------------------------------------- */
void orc_encode(int64_t n, const float *z, int32_t nthr, const float *thr, uint8_t *out)
{
    for (int64_t i = 0; i < n; ++i) {
        int lvl = 0;
        for (int32_t j = 0; j < nthr; ++j) lvl += z[i] > thr[j];
        out[i] = (uint8_t)lvl;
    }
}

/* ------------------------------------------------------------------------------------
 * DM-scaled width set (Methods, "Matched filtering", the equation for W(d_k)): the widths of
 * row k are the base set (the first n_base entries of the increasing width list) and every
 * further width w with w <= alpha * tau_sweep(d_k) / dt, tau_sweep being the dispersive sweep
 * across the band at d_k: the unrounded delay of the lowest channel frequency, evaluated
 * exactly as the channel delays are.  Since the list increases, row k uses its first
 * count[k] widths.  n_base <= 0 keeps every width in every row.
 * ---------------------------------------------------------------------------------- */
int orc_dm_width_counts(int32_t nchan, const double *freq, double tsamp_s, double fref, int32_t ndm,
                        const double *dm, int32_t nw, const int32_t *widths, int32_t n_base, double alpha,
                        int32_t *count)
{
    double fmax = freq[0], fmin = freq[0];
    for (int32_t c = 1; c < nchan; ++c) {
        if (freq[c] > fmax) fmax = freq[c];
        if (freq[c] < fmin) fmin = freq[c];
    }
    double fr = fref > 0.0 ? fref : fmax;
    if (fr < fmax) return -1;
    double tms = tsamp_s * 1e3;
    for (int32_t k = 0; k < ndm; ++k) {
        if (n_base <= 0 || n_base >= nw) {
            count[k] = nw;
            continue;
        }
        double x = ORC_KDM * dm[k];
        x = x * (1.0 / (fmin * fmin) - 1.0 / (fr * fr));
        x = x / tms;  /* tau_sweep / dt in samples */
        double lim = alpha * x;
        int32_t n = n_base;
        for (int32_t i = n_base; i < nw; ++i)
            if ((double)widths[i] <= lim) n = i + 1;
        count[k] = n;
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Boxcar matched filter (Methods, "Matched filtering"): per row the mean and population
 * standard deviation of the valid samples, an optional floor sigma_min on sigma, and for
 * every width W that fits, SNR(k,t,W) = (sum_{t'=t}^{t+W-1} y - mu W) / (sigma sqrt W).
 * The plane holds the maximum over widths (first width on ties; widths must increase)
 * and the index of that width; cells where no width fits hold 0 and -1.  A row with
 * sigma = 0 has S/N 0.  integer_plane = 1 takes mu and sigma from the exact integer sums
 * S1 = sum y, S2 = sum y^2 through one fixed FP64 expression: mu = S1/n,
 * sigma = sqrt(n*S2 - S1*S1)/n with each product and the difference rounded once (exact
 * for 8-bit planes, where every term is an integer below 2^53).
 * ---------------------------------------------------------------------------------- */
int orc_matched_filter_sigma(int32_t integer_plane, int64_t ndm, int64_t nout, const double *y, int32_t nw,
                             const int32_t *widths, const int32_t *row_nw, const double *sigma_in, double sigma_min,
                             double *snr, int32_t *widx, double *mu_out, double *sigma_out);

int orc_matched_filter_rows(int32_t integer_plane, int64_t ndm, int64_t nout, const double *y, int32_t nw,
                            const int32_t *widths, const int32_t *row_nw, double sigma_min, double *snr,
                            int32_t *widx, double *mu_out, double *sigma_out)
{
    return orc_matched_filter_sigma(integer_plane, ndm, nout, y, nw, widths, row_nw, NULL, sigma_min, snr, widx,
                                    mu_out, sigma_out);
}

int orc_matched_filter(int32_t integer_plane, int64_t ndm, int64_t nout, const double *y, int32_t nw,
                       const int32_t *widths, double sigma_min, double *snr, int32_t *widx, double *mu_out,
                       double *sigma_out)
{
    return orc_matched_filter_rows(integer_plane, ndm, nout, y, nw, widths, NULL, sigma_min, snr, widx, mu_out,
                                   sigma_out);
}

/* The same with row k restricted to its first row_nw[k] widths (row_nw NULL: all widths), and
 * sigma of row k given as sigma_in[k] instead of the standard deviation (sigma_in NULL: the
 * standard deviation); the floor sigma_min applies either way. */
int orc_matched_filter_sigma(int32_t integer_plane, int64_t ndm, int64_t nout, const double *y, int32_t nw,
                             const int32_t *widths, const int32_t *row_nw, const double *sigma_in, double sigma_min,
                             double *snr, int32_t *widx, double *mu_out, double *sigma_out)
{
    for (int32_t i = 0; i < nw; ++i)
        if (widths[i] < 1 || (i > 0 && widths[i] <= widths[i - 1])) return -1;
    for (int64_t k = 0; k < ndm; ++k) {
        const double *row = y + k * nout;
        double mu, sigma;
        if (integer_plane) {
            int64_t s1 = 0, s2 = 0;
            for (int64_t t = 0; t < nout; ++t) {
                int64_t v = (int64_t)row[t];
                s1 += v;
                s2 += v * v;
            }
            mu = (double)s1 / (double)nout;
            double num = (double)nout * (double)s2 - (double)s1 * (double)s1;
            sigma = num > 0.0 ? sqrt(num) / (double)nout : 0.0;
        } else {
            double s = 0.0;
            for (int64_t t = 0; t < nout; ++t) s += row[t];
            mu = s / (double)nout;
            double q = 0.0;
            for (int64_t t = 0; t < nout; ++t) q += (row[t] - mu) * (row[t] - mu);
            sigma = sqrt(q / (double)nout);
        }
        if (sigma_in) sigma = sigma_in[k];
        if (sigma < sigma_min) sigma = sigma_min;
        if (mu_out) mu_out[k] = mu;
        if (sigma_out) sigma_out[k] = sigma;
        const int32_t nwk = row_nw ? row_nw[k] : nw;
        for (int64_t t = 0; t < nout; ++t) {
            double best = 0.0;
            int32_t bi = -1;
            for (int32_t i = 0; i < nwk; ++i) {
                int32_t w = widths[i];
                if (t + w > nout) break;
                double s = 0.0;
                for (int32_t j = 0; j < w; ++j) s += row[t + j];
                double val = 0.0;
                if (sigma > 0.0) {
                    double num = s - mu * (double)w;
                    double den = sigma * sqrt((double)w);
                    val = num / den;
                }
                if (bi < 0 || val > best) { best = val; bi = i; }
            }
            snr[k * nout + t] = best;
            widx[k * nout + t] = bi;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Candidate detection (Methods, "Candidate detection"): threshold the S/N plane at
 * theta (S/N >= theta), binary closing with a (2r+1)^2 square evaluated on the
 * zero-extended infinite plane, 8-connected labelling of the closed mask, islands with
 * fewer than n_min pixels dropped, one candidate per island at its peak pixel (highest
 * S/N, then smallest DM index, then smallest time).  Candidates are returned ordered by
 * (DM index, time) of the peak.  Returns the number of candidates found (which may
 * exceed cap; only cap are written) or -1.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int32_t k;
    int32_t widx;
    int64_t t;
    double snr;
    int64_t npix;
} orc_cand;

static int cmp_cand(const void *a, const void *b)
{
    const orc_cand *x = a, *y = b;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    return x->t < y->t ? -1 : x->t > y->t;
}

int64_t orc_candidates(int64_t ndm, int64_t nout, const double *snr, const int32_t *widx, double theta,
                       int32_t r, int64_t n_min, orc_cand *out, int64_t cap)
{
    if (r < 0) return -1;
    int64_t m = 2 * (int64_t)r;
    int64_t H = ndm + 2 * m, W = nout + 2 * m;
    uint8_t *a = calloc((size_t)(H * W), 1), *b = calloc((size_t)(H * W), 1);
    if (!a || !b) { free(a); free(b); return -1; }
    for (int64_t k = 0; k < ndm; ++k)
        for (int64_t t = 0; t < nout; ++t) a[(k + m) * W + t + m] = snr[k * nout + t] >= theta;
    /* dilation: along time, then along DM */
    for (int64_t i = 0; i < H; ++i)
        for (int64_t j = 0; j < W; ++j) {
            uint8_t v = 0;
            for (int64_t d = -r; d <= r && !v; ++d) { int64_t jj = j + d; if (jj >= 0 && jj < W) v = a[i * W + jj]; }
            b[i * W + j] = v;
        }
    for (int64_t i = 0; i < H; ++i)
        for (int64_t j = 0; j < W; ++j) {
            uint8_t v = 0;
            for (int64_t d = -r; d <= r && !v; ++d) { int64_t ii = i + d; if (ii >= 0 && ii < H) v = b[ii * W + j]; }
            a[i * W + j] = v;
        }
    /* erosion: outside the padded array counts as zero, which never matters because the
     * padding (2r) keeps every dilated pixel at least r away from the border */
    for (int64_t i = 0; i < H; ++i)
        for (int64_t j = 0; j < W; ++j) {
            uint8_t v = 1;
            for (int64_t d = -r; d <= r && v; ++d) { int64_t jj = j + d; v = (jj >= 0 && jj < W) ? a[i * W + jj] : 0; }
            b[i * W + j] = v;
        }
    for (int64_t i = 0; i < H; ++i)
        for (int64_t j = 0; j < W; ++j) {
            uint8_t v = 1;
            for (int64_t d = -r; d <= r && v; ++d) { int64_t ii = i + d; v = (ii >= 0 && ii < H) ? b[ii * W + j] : 0; }
            a[i * W + j] = v;
        }
    /* 8-connected labelling of the closed mask, cropped back to the plane */
    uint8_t *seen = calloc((size_t)(ndm * nout), 1);
    int64_t *stack = malloc(sizeof(int64_t) * (size_t)(ndm * nout > 0 ? ndm * nout : 1));
    int64_t ncand = 0, nkept = 0;
    orc_cand *all = NULL;
    for (int64_t k = 0; k < ndm; ++k)
        for (int64_t t = 0; t < nout; ++t) {
            int64_t idx = k * nout + t;
            if (seen[idx] || !a[(k + m) * W + t + m]) continue;
            int64_t sp = 0, npix = 0;
            stack[sp++] = idx;
            seen[idx] = 1;
            orc_cand c = {(int32_t)k, widx[idx], t, snr[idx], 0};
            while (sp) {
                int64_t q = stack[--sp];
                int64_t qk = q / nout, qt = q % nout;
                ++npix;
                double s = snr[q];
                if (s > c.snr || (s == c.snr && (qk < c.k || (qk == c.k && qt < c.t)))) {
                    c.snr = s; c.k = (int32_t)qk; c.t = qt; c.widx = widx[q];
                }
                for (int64_t dk = -1; dk <= 1; ++dk)
                    for (int64_t dt = -1; dt <= 1; ++dt) {
                        int64_t nk = qk + dk, nt2 = qt + dt;
                        if (nk < 0 || nk >= ndm || nt2 < 0 || nt2 >= nout) continue;
                        int64_t ni = nk * nout + nt2;
                        if (!seen[ni] && a[(nk + m) * W + nt2 + m]) { seen[ni] = 1; stack[sp++] = ni; }
                    }
            }
            c.npix = npix;
            ++ncand;
            if (npix < n_min) continue;
            all = realloc(all, sizeof(orc_cand) * (size_t)(nkept + 1));
            all[nkept++] = c;
        }
    (void)ncand;
    if (nkept > 1) qsort(all, (size_t)nkept, sizeof(orc_cand), cmp_cand);
    for (int64_t i = 0; i < nkept && i < cap; ++i) out[i] = all[i];
    free(all); free(seen); free(stack); free(a); free(b);
    return nkept;
}

/* ------------------------------------------------------------------------------------
 * Front-end RFI steps (Results, "False-positive rate": windowed MAD channel flagging and
 * optional zero-DM subtraction; Table S1: gamma_zdm).  z is a z-scored filterbank
 * [nchan][n] of float32, changed in place.
 *
 * Zero-DM: S(t) = sum over channels in order (FP64); where |S(t)| / sqrt(nchan) > gamma every
 * channel becomes (float)(z - S(t) / nchan).  Returns the number of samples changed.
 * ---------------------------------------------------------------------------------- */
int64_t orc_zero_dm(int32_t nchan, int64_t n, float *z, double gamma)
{
    int64_t changed = 0;
    for (int64_t t = 0; t < n; ++t) {
        double s = 0.0;
        for (int32_t c = 0; c < nchan; ++c) s += (double)z[(int64_t)c * n + t];
        if (fabs(s) / sqrt((double)nchan) > gamma) {
            double mean = s / (double)nchan;
            for (int32_t c = 0; c < nchan; ++c) z[(int64_t)c * n + t] = (float)((double)z[(int64_t)c * n + t] - mean);
            ++changed;
        }
    }
    return changed;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Lower median: element floor((n - 1) / 2) of the sorted values. */
static double lower_median(const double *v, int32_t n, double *scratch)
{
    memcpy(scratch, v, (size_t)n * sizeof(double));
    qsort(scratch, (size_t)n, sizeof(double), cmp_double);
    return scratch[(n - 1) / 2];
}

/* Sum of v[0..len) (squared deviations from `shift` when `squared`), one FP64 accumulator
 * taking the samples in time order: the plain definition of the sum, no partial sums. */
static double window_sum(const float *v, int64_t len, double shift, int squared)
{
    double s = 0.0;
    for (int64_t t = 0; t < len; ++t) {
        double x = (double)v[t] - shift;
        s += squared ? x * x : x;
    }
    return s;
}

/* Channel flagging (Results, "False-positive rate": windowed MAD channel flagging): per window
 * of w samples (the last may be shorter), s_c = population standard deviation of channel c over
 * the window (two passes: the mean, then the mean squared deviation from it, each a plain FP64
 * sum in time order); m = lower median of s, mad = lower median of
 * |s_c - m|; channel c is flagged when |s_c - m| > k * (mad_scale * mad) and its window samples
 * are set to 0.  flags [nwin][nchan] receives 1 / 0, sigma_out [nwin][nchan] the s_c (may be
 * NULL).  Returns 0, or -1 when memory runs out. */
int orc_flag_channels(int32_t nchan, int64_t n, float *z, int64_t w, double k, double mad_scale, uint8_t *flags,
                      double *sigma_out)
{
    double *s = malloc((size_t)nchan * sizeof(double)), *d = malloc((size_t)nchan * sizeof(double));
    double *tmp = malloc((size_t)nchan * sizeof(double));
    if (!s || !d || !tmp) { free(s); free(d); free(tmp); return -1; }
    int64_t nwin = (n + w - 1) / w;
    for (int64_t b = 0; b < nwin; ++b) {
        int64_t t0 = b * w, len = n - t0 < w ? n - t0 : w;
        for (int32_t c = 0; c < nchan; ++c) {
            const float *row = z + (int64_t)c * n + t0;
            double mu = window_sum(row, len, 0.0, 0) / (double)len;
            s[c] = sqrt(window_sum(row, len, mu, 1) / (double)len);
            if (sigma_out) sigma_out[b * nchan + c] = s[c];
        }
        double m = lower_median(s, nchan, tmp);
        for (int32_t c = 0; c < nchan; ++c) d[c] = fabs(s[c] - m);
        double thr = k * (mad_scale * lower_median(d, nchan, tmp));
        for (int32_t c = 0; c < nchan; ++c) {
            int f = d[c] > thr;
            flags[b * nchan + c] = (uint8_t)f;
            if (f)
                for (int64_t t = 0; t < len; ++t) z[(int64_t)c * n + t0 + t] = 0.0f;
        }
    }
    free(s);
    free(d);
    free(tmp);
    return 0;
}
