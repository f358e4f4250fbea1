/*
 * CPU oracle for maximal biclique enumeration (MBE).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * Two independent routes to the same set
 *     B(G) = { (A, B) : A subset of U, B subset of V, both non-empty, B = N(A), A = N(B) },
 * the maximal bicliques of the bipartite graph G = (U u V, E) (paper, section II-A,
 * definition of biclique, maximality and common neighbours N(X)):
 *
 *   orc_brute  -- the definition written out: every non-empty A subset of U (|U| <= 24,
 *                 |V| <= 64), B = N(A), keep the pair when B is non-empty and N(B) = A.
 *   orc_mbea   -- MBEA as the paper states it (Algorithm 1, section II-B), serial and
 *                 recursive, on sorted vertex lists, with the reverse-scanning count of
 *                 section III-E for |N(v) n L'| and the candidate order of sections II-C
 *                 and III-E (ascending common-neighbour count).
 *
 * Letters.  Algorithm 1 grows R (a subset of U) and shrinks L (a subset of V).  This file
 * uses the opposite letters, which the library uses too: the candidate vertex joins the
 * growing set L, and the shrinking set R is intersected with its neighbour list.  The
 * candidate side C holds L, P and Q; the other side O holds R.
 *
 * Readings of the paper taken here (each is also listed in the design notes):
 *   r1  both sides of a reported biclique are non-empty (section II-A is silent);
 *   r2  the top call is MBEA(L = {}, R = O, P = {v in C : deg v > 0}, Q = {}), since a
 *       degree-0 candidate would be reported with an empty side;
 *   r3  L', R', P', Q' are reset for every candidate x (Algorithm 1 initialises them once);
 *   r4  C is the smaller side, U on a tie (the paper assumes |V| >= |U| with P in U);
 *   r5  P is processed in ascending |N(v) n R|, ties kept in the order the vertices had in
 *       the parent's candidate list (a stable sort); at the top level the key is deg v and
 *       ties go by ascending vertex id; a child's P' is built by walking the rest of P in
 *       order and is then stably sorted by the counts found while building it;
 *   r6  a candidate v enters P' when 0 < |N(v) n R'| < |R'| (Algorithm 1, expansion step;
 *       the fine-grained section prints the inequality garbled);
 *   r7  the hash of a biclique follows the SplitMix64 output function (see orc_hash_pair);
 *   r13 the pivot rule of orc_pivot (see pivot_mbea): one pivot per list below the top
 *       level, the first candidate of the largest count, covering by containment within R.
 *
 * Diagnostics (nodes, non-maximal nodes, depth, algorithmic bytes) follow the same tree.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ hash (reading r7) */

/* SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014), mod 2^64. */
static uint64_t orc_mix(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

#define ORC_K 0x9E3779B97F4A7C15ULL

uint64_t orc_mix64(uint64_t z) { return orc_mix(z); }

/* hu(a) = mix(K (2a+1)) for a in U, hv(b) = mix(K (2b+2)) for b in V. */
static uint64_t orc_hu(int32_t a) { return orc_mix(ORC_K * (2ULL * (uint64_t)a + 1ULL)); }
static uint64_t orc_hv(int32_t b) { return orc_mix(ORC_K * (2ULL * (uint64_t)b + 2ULL)); }

/* The per-vertex terms, exported so that tests can pin them against the published SplitMix64
 * outputs: hu(a) is output 2a+1 and hv(b) output 2b+2 of the generator started from state 0. */
uint64_t orc_hash_u(int32_t a) { return orc_hu(a); }
uint64_t orc_hash_v(int32_t b) { return orc_hv(b); }

/* h(A, B) = mix(sum hu(A) + mix(sum hv(B) + K)); A in U, B in V (caller orientation). */
uint64_t orc_hash_pair(const int32_t *a, int64_t na, const int32_t *b, int64_t nb) {
    uint64_t sa = 0, sb = 0;
    for (int64_t i = 0; i < na; i++) sa += orc_hu(a[i]);
    for (int64_t i = 0; i < nb; i++) sb += orc_hv(b[i]);
    return orc_mix(sa + orc_mix(sb + ORC_K));
}

/* ------------------------------------------------------------------ result record */

typedef struct {
    uint64_t count;      /* |B(G)| restricted to the processed top-level candidates */
    uint64_t hash;       /* sum of h(A, B), mod 2^64 */
    uint64_t out_ints;   /* sum of 2 + |A| + |B| */
    uint64_t nodes;      /* candidates x taken (one per while-iteration of Algorithm 1) */
    uint64_t nonmaximal; /* candidates whose maximality check failed */
    uint64_t bytes_alg;  /* algorithmic bytes, see node_bytes below */
    uint64_t bytes_rs;   /* the same with the reverse-scan term only */
    uint32_t max_depth;  /* deepest level at which a candidate was taken (top level = 1) */
    uint32_t side;       /* 1: C = U, 2: C = V */
    int64_t  written;    /* ints written to the record buffer (-1 if it overflowed) */
} orc_result;

/* ------------------------------------------------------------------ the search */

typedef struct { int32_t key; int32_t v; int32_t seq; } orc_cand;

typedef struct {
    int32_t nc, no;
    const int32_t *c_off, *c_adj;   /* N(v) for v in C: ascending ids in O */
    const int32_t *o_off, *o_adj;   /* N(w) for w in O: ascending ids in C */
    int c_is_v;                     /* candidate side is V: report (R, L) as (A, B) */
    int32_t *cnt;                   /* |N(v) n R'| scratch, all zero between nodes */
    int32_t *buf;                   /* optional record output */
    int64_t buf_cap;
    orc_result *res;
    int32_t *tmp_a, *tmp_b;         /* sorted copies for records */
} orc_ctx;

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* ascending key; equal keys keep their construction order (seq), which makes qsort stable */
static int cmp_cand(const void *a, const void *b) {
    const orc_cand *x = (const orc_cand *)a, *y = (const orc_cand *)b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->seq > y->seq) - (x->seq < y->seq);
}

static int64_t deg_c(const orc_ctx *g, int32_t v) { return g->c_off[v + 1] - g->c_off[v]; }
static int64_t deg_o(const orc_ctx *g, int32_t w) { return g->o_off[w + 1] - g->o_off[w]; }

/* R' = R n N(x): both ascending; walk them together, or binary-search the short list in
 * the long one when the lengths differ a lot.  Returns |R'|. */
static int32_t intersect(const int32_t *r, int32_t nr, const int32_t *nx, int32_t nn, int32_t *out) {
    int32_t k = 0;
    if ((int64_t)nr > 16 * (int64_t)nn) {
        for (int32_t j = 0; j < nn; j++) {
            int32_t lo = 0, hi = nr;
            while (lo < hi) { int32_t mid = lo + (hi - lo) / 2; if (r[mid] < nx[j]) lo = mid + 1; else hi = mid; }
            if (lo < nr && r[lo] == nx[j]) out[k++] = nx[j];
        }
        return k;
    }
    int32_t i = 0, j = 0;
    while (i < nr && j < nn) {
        if (r[i] < nx[j]) i++;
        else if (r[i] > nx[j]) j++;
        else { out[k++] = r[i]; i++; j++; }
    }
    return k;
}

static void report(orc_ctx *g, const int32_t *l, int32_t nl, const int32_t *r, int32_t nr) {
    /* caller orientation: A in U, B in V */
    const int32_t *a = g->c_is_v ? r : l, *b = g->c_is_v ? l : r;
    int32_t na = g->c_is_v ? nr : nl, nb = g->c_is_v ? nl : nr;
    orc_result *res = g->res;
    res->count += 1;
    res->hash += orc_hash_pair(a, na, b, nb);
    res->out_ints += 2 + (uint64_t)na + (uint64_t)nb;
    if (g->buf && res->written >= 0) {
        if (res->written + 2 + na + nb > g->buf_cap) { res->written = -1; return; }
        int32_t *o = g->buf + res->written;
        o[0] = na; o[1] = nb;
        memcpy(o + 2, a, sizeof(int32_t) * (size_t)na);
        memcpy(o + 2 + na, b, sizeof(int32_t) * (size_t)nb);
        qsort(o + 2, (size_t)na, sizeof(int32_t), cmp_i32);
        qsort(o + 2 + na, (size_t)nb, sizeof(int32_t), cmp_i32);
        res->written += 2 + na + nb;
    }
}

/*
 * One call of Algorithm 1 (MBEA(L, R, P, Q)) in this file's letters.
 *   L: the growing set (candidate side), R: the shrinking set (other side, ascending),
 *   P: candidates in processing order (reading r5), Q: the maximality-check set.
 * P and Q are owned by the caller; Q gains each tested x (last step of the loop body), so
 * it is passed with room for |Q| + |P| entries.
 */
static void mbea(orc_ctx *g, const int32_t *L, int32_t nL, const int32_t *R, int32_t nR,
                 const orc_cand *P, int32_t nP, int32_t *Q, int32_t nQ, uint32_t depth,
                 int32_t stop_after) {
    if (depth > g->res->max_depth) g->res->max_depth = depth;
    int32_t *Lp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nL + nP + 1));
    int32_t *Rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nR + 1));
    orc_cand *Pp = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(nP + 1));
    int32_t *Qp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nQ + nP + 1));
    int32_t taken = 0;

    for (int32_t ip = 0; ip < nP; ip++) {           /* while |P| > 0 */
        if (stop_after >= 0 && taken >= stop_after) break;
        taken++;
        /* Step 1, candidate selection: x = P.pop(), the next in order (reading r5) */
        int32_t x = P[ip].v;
        const orc_cand *Prest = P + ip + 1;
        int32_t nPrest = nP - ip - 1;
        g->res->nodes += 1;

        /* L' = L u {x} (reading r3: L', R', P', Q' start afresh for each x) */
        int32_t nLp = 0;
        for (int32_t i = 0; i < nL; i++) Lp[nLp++] = L[i];
        Lp[nLp++] = x;

        /* Step 2, R' construction: R' = R n N(x) */
        const int32_t *nx = g->c_adj + g->c_off[x];
        int32_t nRp = intersect(R, nR, nx, (int32_t)deg_c(g, x), Rp);

        /* |N(v) n R'| for every v by reverse scanning (section III-E): walk each w in R'
         * and its neighbours, adding one to the count of each neighbour */
        for (int32_t i = 0; i < nRp; i++) {
            int32_t w = Rp[i];
            for (int32_t e = g->o_off[w]; e < g->o_off[w + 1]; e++) g->cnt[g->o_adj[e]] += 1;
        }

        /* algorithmic bytes of this node: x's row, the cheaper containment-scan direction,
         * the node's set state and the child's */
        uint64_t rs = 0, fw = 0;
        for (int32_t i = 0; i < nRp; i++) rs += 2 + (uint64_t)deg_o(g, Rp[i]);
        for (int32_t i = 0; i < nPrest; i++) fw += 2 + (uint64_t)deg_c(g, Prest[i].v);
        for (int32_t i = 0; i < nQ; i++) fw += 2 + (uint64_t)deg_c(g, Q[i]);

        /* Step 3, maximality checking against Q */
        int maximal = 1;
        int32_t nQp = 0;
        for (int32_t i = 0; i < nQ; i++) {
            int32_t c = g->cnt[Q[i]];
            if (c == nRp) { maximal = 0; break; }
            else if (c > 0) Qp[nQp++] = Q[i];
        }

        int32_t nPp = 0;
        if (maximal) {
            /* Step 4, maximal expansion over the rest of P */
            for (int32_t i = 0; i < nPrest; i++) {
                int32_t v = Prest[i].v, c = g->cnt[v];
                if (c == nRp) Lp[nLp++] = v;
                else if (c > 0) { Pp[nPp].key = c; Pp[nPp].v = v; Pp[nPp].seq = nPp; nPp++; }
            }
        } else {
            g->res->nonmaximal += 1;
            nQp = 0;
        }

        /* counts back to zero before anything else uses them */
        for (int32_t i = 0; i < nRp; i++) {
            int32_t w = Rp[i];
            for (int32_t e = g->o_off[w]; e < g->o_off[w + 1]; e++) g->cnt[g->o_adj[e]] = 0;
        }

        uint64_t state = (uint64_t)nPrest + (uint64_t)nQ + (uint64_t)nRp + (uint64_t)nPp + (uint64_t)nQp;
        uint64_t base = 2 + (uint64_t)deg_c(g, x) + state;
        g->res->bytes_alg += 4 * (base + (rs < fw ? rs : fw));
        g->res->bytes_rs += 4 * (base + rs);

        if (maximal) {
            report(g, Lp, nLp, Rp, nRp);                 /* B = B u {(L', R')} */
            if (nPp > 0) {
                qsort(Pp, (size_t)nPp, sizeof(orc_cand), cmp_cand);
                int32_t *Qchild = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nQp + nPp + 1));
                memcpy(Qchild, Qp, sizeof(int32_t) * (size_t)nQp);
                mbea(g, Lp, nLp, Rp, nRp, Pp, nPp, Qchild, nQp, depth + 1, -1);
                free(Qchild);
            }
        }
        Q[nQ++] = x;                                    /* Q = Q u {x} */
    }
    free(Lp); free(Rp); free(Pp); free(Qp);
}

/* |R n N(v)| for ascending R and N(v) (a count-only merge). */
static int32_t meet_count(const int32_t *r, int32_t nr, const int32_t *nv, int32_t nn) {
    int32_t i = 0, j = 0, k = 0;
    while (i < nr && j < nn) {
        if (r[i] < nv[j]) i++;
        else if (r[i] > nv[j]) j++;
        else { k++; i++; j++; }
    }
    return k;
}

/*
 * Algorithm 1 with iMBEA's candidate pruning (the embedded pruning of section II-C, after
 * Zhang et al.): when x's node is maximal, every other candidate v of P that joins L' (it is
 * adjacent to all of R') and has no neighbour in R outside R' -- so its neighbourhood within
 * R is exactly x's -- leaves P and joins Q together with x.  Such a v could only head nodes
 * whose bicliques x's subtree already holds, so the answer is the same with fewer nodes.
 * When x is not maximal nothing else moves (the maximal-expansion scan is where the test is
 * made).  A candidate that has left P is never taken; for the nodes after x it is in Q.
 *
 * silent_before: candidates at positions below it are only run for their effect on P and Q
 * (maximality, and the set that leaves P with them), with nothing counted or reported and no
 * recursion -- the top-level prefix of a rank range, so that a range sees the moves the whole
 * run makes.  stop_before: positions from here on are not taken.
 */
static void imbea(orc_ctx *g, const int32_t *L, int32_t nL, const int32_t *R, int32_t nR,
                  const orc_cand *P, int32_t nP, int32_t *Q, int32_t nQ, uint32_t depth,
                  int32_t silent_before, int32_t stop_before) {
    int32_t *Lp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nL + nP + 1));
    int32_t *Rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nR + 1));
    orc_cand *Pp = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(nP + 1));
    int32_t *Qp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nQ + nP + 1));
    int32_t *Cs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nP + 1));   /* positions leaving P */
    unsigned char *gone = (unsigned char *)calloc((size_t)nP + 1, 1);

    for (int32_t ip = 0; ip < nP && ip < stop_before; ip++) {
        if (gone[ip]) continue;                          /* left P with an earlier x */
        const int silent = ip < silent_before;
        int32_t x = P[ip].v;
        if (!silent) {
            g->res->nodes += 1;
            if (depth > g->res->max_depth) g->res->max_depth = depth;
        }
        int32_t nLp = 0;
        for (int32_t i = 0; i < nL; i++) Lp[nLp++] = L[i];
        Lp[nLp++] = x;
        const int32_t *nx = g->c_adj + g->c_off[x];
        int32_t nRp = intersect(R, nR, nx, (int32_t)deg_c(g, x), Rp);
        for (int32_t i = 0; i < nRp; i++) {
            int32_t w = Rp[i];
            for (int32_t e = g->o_off[w]; e < g->o_off[w + 1]; e++) g->cnt[g->o_adj[e]] += 1;
        }
        /* the same byte tally as the plain search, over the P and Q of this moment */
        uint64_t rs = 0, fw = 0, nPrest = 0;
        for (int32_t i = 0; i < nRp; i++) rs += 2 + (uint64_t)deg_o(g, Rp[i]);
        for (int32_t i = ip + 1; i < nP; i++)
            if (!gone[i]) { fw += 2 + (uint64_t)deg_c(g, P[i].v); nPrest++; }
        for (int32_t i = 0; i < nQ; i++) fw += 2 + (uint64_t)deg_c(g, Q[i]);

        int maximal = 1;
        int32_t nQp = 0;
        for (int32_t i = 0; i < nQ; i++) {
            int32_t c = g->cnt[Q[i]];
            if (c == nRp) { maximal = 0; break; }
            else if (c > 0) Qp[nQp++] = Q[i];
        }
        int32_t nPp = 0, nC = 0;
        if (maximal) {
            for (int32_t i = ip + 1; i < nP; i++) {
                if (gone[i]) continue;
                int32_t v = P[i].v, c = g->cnt[v];
                if (c == nRp) {
                    Lp[nLp++] = v;
                    /* v joins L'; with no neighbour in R outside R' it also leaves P */
                    if (meet_count(R, nR, g->c_adj + g->c_off[v], (int32_t)deg_c(g, v)) == nRp) Cs[nC++] = i;
                } else if (c > 0) { Pp[nPp].key = c; Pp[nPp].v = v; Pp[nPp].seq = nPp; nPp++; }
            }
        } else {
            if (!silent) g->res->nonmaximal += 1;
            nQp = 0;
        }
        for (int32_t i = 0; i < nRp; i++) {
            int32_t w = Rp[i];
            for (int32_t e = g->o_off[w]; e < g->o_off[w + 1]; e++) g->cnt[g->o_adj[e]] = 0;
        }
        if (!silent) {
            uint64_t state = nPrest + (uint64_t)nQ + (uint64_t)nRp + (uint64_t)nPp + (uint64_t)nQp;
            uint64_t base = 2 + (uint64_t)deg_c(g, x) + state;
            g->res->bytes_alg += 4 * (base + (rs < fw ? rs : fw));
            g->res->bytes_rs += 4 * (base + rs);
        }
        if (maximal && !silent) {
            report(g, Lp, nLp, Rp, nRp);
            if (nPp > 0) {
                qsort(Pp, (size_t)nPp, sizeof(orc_cand), cmp_cand);
                int32_t *Qchild = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nQp + nPp + 1));
                memcpy(Qchild, Qp, sizeof(int32_t) * (size_t)nQp);
                imbea(g, Lp, nLp, Rp, nRp, Pp, nPp, Qchild, nQp, depth + 1, 0, nPp);
                free(Qchild);
            }
        }
        Q[nQ++] = x;                                     /* Q = Q u C, C = {x} u the moved */
        for (int32_t k = 0; k < nC; k++) {
            gone[Cs[k]] = 1;
            Q[nQ++] = P[Cs[k]].v;
        }
    }
    free(Lp); free(Rp); free(Pp); free(Qp); free(Cs); free(gone);
}

/*
 * Algorithm 1 with a pivot rule: the pivot pruning that section II-C describes (after PMBEA's
 * containment of neighbourhoods, NCR), in the reading this file takes (r13).  In every list
 * below the top level, the candidate p with the largest |N(p) n R| (the first such in the
 * list's order) is taken first, and every other candidate v whose neighbours within R are all
 * neighbours of p (N(v) n R a subset of N(p) n R) is covered by p: a maximal biclique whose L
 * holds v holds p as well, so p's subtree finds it and v is never taken at this node.  The list
 * is regrouped as p, then the candidates p covers, then the others (each group in the list's
 * order), and the loop of Algorithm 1 runs over the regrouped list with the covered
 * candidates passed over: they are candidates for p's node and, like every entry the loop has
 * passed, Q entries for the nodes after them.  The top-level list keeps its order (its
 * candidates are the independent root tasks of section III-C).
 */
static void pivot_mbea(orc_ctx *g, const int32_t *L, int32_t nL, const int32_t *R, int32_t nR,
                       const orc_cand *P0, int32_t nP, int32_t *Q, int32_t nQ, uint32_t depth,
                       int32_t stop_after) {
    orc_cand *P = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(nP + 1));
    unsigned char *covered = (unsigned char *)calloc((size_t)nP + 1, 1);
    if (depth == 1 || nP < 2) {
        memcpy(P, P0, sizeof(orc_cand) * (size_t)nP);
    } else {
        int32_t ip = 0;
        for (int32_t i = 1; i < nP; i++)
            if (P0[i].key > P0[ip].key) ip = i;             /* the first of the largest count */
        const int32_t pv = P0[ip].v;
        int32_t *Np = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nR + 1));
        int32_t nNp = intersect(R, nR, g->c_adj + g->c_off[pv], (int32_t)deg_c(g, pv), Np);
        unsigned char *in = (unsigned char *)calloc((size_t)nP + 1, 1);
        for (int32_t i = 0; i < nP; i++) {
            if (i == ip) continue;
            const int32_t *nv = g->c_adj + g->c_off[P0[i].v];
            int32_t dv = (int32_t)deg_c(g, P0[i].v);
            /* N(v) n R inside N(p) n R: v meets N(p) n R as often as it meets R */
            in[i] = meet_count(Np, nNp, nv, dv) == meet_count(R, nR, nv, dv);
        }
        int32_t k = 0;
        P[k++] = P0[ip];
        for (int32_t i = 0; i < nP; i++)
            if (i != ip && in[i]) { covered[k] = 1; P[k++] = P0[i]; }
        for (int32_t i = 0; i < nP; i++)
            if (i != ip && !in[i]) P[k++] = P0[i];
        free(Np); free(in);
    }
    int32_t *Lp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nL + nP + 1));
    int32_t *Rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nR + 1));
    orc_cand *Pp = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(nP + 1));
    int32_t *Qp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nQ + nP + 1));
    int32_t taken = 0;

    for (int32_t ip = 0; ip < nP; ip++) {
        if (stop_after >= 0 && taken >= stop_after) break;
        int32_t x = P[ip].v;
        if (covered[ip]) { Q[nQ++] = x; continue; }      /* passed over: a Q entry from here on */
        taken++;
        const orc_cand *Prest = P + ip + 1;
        int32_t nPrest = nP - ip - 1;
        g->res->nodes += 1;
        if (depth > g->res->max_depth) g->res->max_depth = depth;
        int32_t nLp = 0;
        for (int32_t i = 0; i < nL; i++) Lp[nLp++] = L[i];
        Lp[nLp++] = x;
        const int32_t *nx = g->c_adj + g->c_off[x];
        int32_t nRp = intersect(R, nR, nx, (int32_t)deg_c(g, x), Rp);
        for (int32_t i = 0; i < nRp; i++) {
            int32_t w = Rp[i];
            for (int32_t e = g->o_off[w]; e < g->o_off[w + 1]; e++) g->cnt[g->o_adj[e]] += 1;
        }
        uint64_t rs = 0, fw = 0;
        for (int32_t i = 0; i < nRp; i++) rs += 2 + (uint64_t)deg_o(g, Rp[i]);
        for (int32_t i = 0; i < nPrest; i++) fw += 2 + (uint64_t)deg_c(g, Prest[i].v);
        for (int32_t i = 0; i < nQ; i++) fw += 2 + (uint64_t)deg_c(g, Q[i]);
        int maximal = 1;
        int32_t nQp = 0;
        for (int32_t i = 0; i < nQ; i++) {
            int32_t c = g->cnt[Q[i]];
            if (c == nRp) { maximal = 0; break; }
            else if (c > 0) Qp[nQp++] = Q[i];
        }
        int32_t nPp = 0;
        if (maximal) {
            for (int32_t i = 0; i < nPrest; i++) {
                int32_t v = Prest[i].v, c = g->cnt[v];
                if (c == nRp) Lp[nLp++] = v;
                else if (c > 0) { Pp[nPp].key = c; Pp[nPp].v = v; Pp[nPp].seq = nPp; nPp++; }
            }
        } else {
            g->res->nonmaximal += 1;
            nQp = 0;
        }
        for (int32_t i = 0; i < nRp; i++) {
            int32_t w = Rp[i];
            for (int32_t e = g->o_off[w]; e < g->o_off[w + 1]; e++) g->cnt[g->o_adj[e]] = 0;
        }
        uint64_t state = (uint64_t)nPrest + (uint64_t)nQ + (uint64_t)nRp + (uint64_t)nPp + (uint64_t)nQp;
        uint64_t base = 2 + (uint64_t)deg_c(g, x) + state;
        g->res->bytes_alg += 4 * (base + (rs < fw ? rs : fw));
        g->res->bytes_rs += 4 * (base + rs);
        if (maximal) {
            report(g, Lp, nLp, Rp, nRp);
            if (nPp > 0) {
                qsort(Pp, (size_t)nPp, sizeof(orc_cand), cmp_cand);
                int32_t *Qchild = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nQp + nPp + 1));
                memcpy(Qchild, Qp, sizeof(int32_t) * (size_t)nQp);
                pivot_mbea(g, Lp, nLp, Rp, nRp, Pp, nPp, Qchild, nQp, depth + 1, -1);
                free(Qchild);
            }
        }
        Q[nQ++] = x;
    }
    free(P); free(covered); free(Lp); free(Rp); free(Pp); free(Qp);
}

/* Candidate side: 1 = U, 2 = V, 0 = the smaller side, U on a tie (reading r4). */
static int pick_side(int32_t n_u, int32_t n_v, int side) {
    if (side == 1 || side == 2) return side;
    return n_v < n_u ? 2 : 1;
}

/*
 * Serial MBEA over the whole graph, or over the top-level candidates whose rank (position
 * in the ascending (deg, id) order) lies in [rank_lo, rank_hi).  Candidates ranked before
 * rank_lo start in Q, so splitting the ranks into ranges and summing the results gives the
 * whole result exactly.  buf (may be NULL) receives records [|A|, |B|, A..., B...] with A
 * in U and B in V, each side ascending, in discovery order.  Returns 0, or -1 on bad
 * arguments or allocation failure.
 */
int orc_mbea(int32_t n_u, int32_t n_v, const int32_t *u_off, const int32_t *u_adj,
             const int32_t *v_off, const int32_t *v_adj, int side, int64_t rank_lo,
             int64_t rank_hi, int32_t *buf, int64_t buf_cap, orc_result *res) {
    if (!res || n_u < 0 || n_v < 0) return -1;
    memset(res, 0, sizeof(*res));
    side = pick_side(n_u, n_v, side);
    res->side = (uint32_t)side;
    orc_ctx g;
    memset(&g, 0, sizeof(g));
    g.c_is_v = (side == 2);
    g.nc = g.c_is_v ? n_v : n_u;
    g.no = g.c_is_v ? n_u : n_v;
    g.c_off = g.c_is_v ? v_off : u_off;
    g.c_adj = g.c_is_v ? v_adj : u_adj;
    g.o_off = g.c_is_v ? u_off : v_off;
    g.o_adj = g.c_is_v ? u_adj : v_adj;
    g.buf = buf;
    g.buf_cap = buf_cap;
    g.res = res;
    if (g.nc == 0 || g.no == 0) return 0;

    /* top-level P: candidates with at least one neighbour, ascending (deg, id) (r2, r5);
     * ids ascend in the scan, so seq = id makes equal degrees keep id order */
    orc_cand *P = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)g.nc);
    int32_t nP = 0;
    for (int32_t v = 0; v < g.nc; v++) {
        int64_t d = deg_c(&g, v);
        if (d > 0) { P[nP].key = (int32_t)d; P[nP].v = v; P[nP].seq = v; nP++; }
    }
    qsort(P, (size_t)nP, sizeof(orc_cand), cmp_cand);
    if (rank_lo < 0) rank_lo = 0;
    if (rank_hi < 0 || rank_hi > nP) rank_hi = nP;
    int32_t *R = (int32_t *)malloc(sizeof(int32_t) * (size_t)g.no);
    for (int32_t w = 0; w < g.no; w++) R[w] = w;   /* R = O */
    int32_t *Q = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nP + 1));
    int32_t nQ = 0;
    for (int64_t i = 0; i < rank_lo && i < nP; i++) Q[nQ++] = P[i].v;
    g.cnt = (int32_t *)calloc((size_t)g.nc, sizeof(int32_t));
    if (!P || !R || !Q || !g.cnt) { free(P); free(R); free(Q); free(g.cnt); return -1; }
    if (rank_lo < rank_hi)
        mbea(&g, NULL, 0, R, g.no, P + rank_lo, (int32_t)(nP - rank_lo), Q, nQ, 1,
             (int32_t)(rank_hi - rank_lo));
    free(P); free(R); free(Q); free(g.cnt);
    return 0;
}

/*
 * As orc_mbea, with iMBEA's candidate pruning (see imbea above).  The top-level candidates
 * ranked before rank_lo are run silently, so that a rank range makes the moves the whole run
 * makes: count, hash and the tree tallies of disjoint ranges add up to the whole run's.
 */
int orc_imbea(int32_t n_u, int32_t n_v, const int32_t *u_off, const int32_t *u_adj,
              const int32_t *v_off, const int32_t *v_adj, int side, int64_t rank_lo,
              int64_t rank_hi, int32_t *buf, int64_t buf_cap, orc_result *res) {
    if (!res || n_u < 0 || n_v < 0) return -1;
    memset(res, 0, sizeof(*res));
    side = pick_side(n_u, n_v, side);
    res->side = (uint32_t)side;
    orc_ctx g;
    memset(&g, 0, sizeof(g));
    g.c_is_v = (side == 2);
    g.nc = g.c_is_v ? n_v : n_u;
    g.no = g.c_is_v ? n_u : n_v;
    g.c_off = g.c_is_v ? v_off : u_off;
    g.c_adj = g.c_is_v ? v_adj : u_adj;
    g.o_off = g.c_is_v ? u_off : v_off;
    g.o_adj = g.c_is_v ? u_adj : v_adj;
    g.buf = buf;
    g.buf_cap = buf_cap;
    g.res = res;
    if (g.nc == 0 || g.no == 0) return 0;
    orc_cand *P = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)g.nc);
    int32_t nP = 0;
    for (int32_t v = 0; v < g.nc; v++) {
        int64_t d = deg_c(&g, v);
        if (d > 0) { P[nP].key = (int32_t)d; P[nP].v = v; P[nP].seq = v; nP++; }
    }
    qsort(P, (size_t)nP, sizeof(orc_cand), cmp_cand);
    if (rank_lo < 0) rank_lo = 0;
    if (rank_hi < 0 || rank_hi > nP) rank_hi = nP;
    int32_t *R = (int32_t *)malloc(sizeof(int32_t) * (size_t)g.no);
    for (int32_t w = 0; w < g.no; w++) R[w] = w;
    int32_t *Q = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nP + 1));
    g.cnt = (int32_t *)calloc((size_t)g.nc, sizeof(int32_t));
    if (!P || !R || !Q || !g.cnt) { free(P); free(R); free(Q); free(g.cnt); return -1; }
    if (rank_lo < rank_hi) imbea(&g, NULL, 0, R, g.no, P, nP, Q, 0, 1, (int32_t)rank_lo, (int32_t)rank_hi);
    free(P); free(R); free(Q); free(g.cnt);
    return 0;
}

/*
 * As orc_mbea, with the pivot rule (see pivot_mbea).  The top-level list keeps the plain
 * order, so rank ranges split the run exactly as they do for orc_mbea.
 */
int orc_pivot(int32_t n_u, int32_t n_v, const int32_t *u_off, const int32_t *u_adj,
              const int32_t *v_off, const int32_t *v_adj, int side, int64_t rank_lo,
              int64_t rank_hi, int32_t *buf, int64_t buf_cap, orc_result *res) {
    if (!res || n_u < 0 || n_v < 0) return -1;
    memset(res, 0, sizeof(*res));
    side = pick_side(n_u, n_v, side);
    res->side = (uint32_t)side;
    orc_ctx g;
    memset(&g, 0, sizeof(g));
    g.c_is_v = (side == 2);
    g.nc = g.c_is_v ? n_v : n_u;
    g.no = g.c_is_v ? n_u : n_v;
    g.c_off = g.c_is_v ? v_off : u_off;
    g.c_adj = g.c_is_v ? v_adj : u_adj;
    g.o_off = g.c_is_v ? u_off : v_off;
    g.o_adj = g.c_is_v ? u_adj : v_adj;
    g.buf = buf;
    g.buf_cap = buf_cap;
    g.res = res;
    if (g.nc == 0 || g.no == 0) return 0;
    orc_cand *P = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)g.nc);
    int32_t nP = 0;
    for (int32_t v = 0; v < g.nc; v++) {
        int64_t d = deg_c(&g, v);
        if (d > 0) { P[nP].key = (int32_t)d; P[nP].v = v; P[nP].seq = v; nP++; }
    }
    qsort(P, (size_t)nP, sizeof(orc_cand), cmp_cand);
    if (rank_lo < 0) rank_lo = 0;
    if (rank_hi < 0 || rank_hi > nP) rank_hi = nP;
    int32_t *R = (int32_t *)malloc(sizeof(int32_t) * (size_t)g.no);
    for (int32_t w = 0; w < g.no; w++) R[w] = w;
    int32_t *Q = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nP + 1));
    int32_t nQ = 0;
    for (int64_t i = 0; i < rank_lo && i < nP; i++) Q[nQ++] = P[i].v;
    g.cnt = (int32_t *)calloc((size_t)g.nc, sizeof(int32_t));
    if (!P || !R || !Q || !g.cnt) { free(P); free(R); free(Q); free(g.cnt); return -1; }
    if (rank_lo < rank_hi)
        pivot_mbea(&g, NULL, 0, R, g.no, P + rank_lo, (int32_t)(nP - rank_lo), Q, nQ, 1,
                   (int32_t)(rank_hi - rank_lo));
    free(P); free(R); free(Q); free(g.cnt);
    return 0;
}

/* Number of top-level candidates (vertices of the candidate side with degree > 0). */
int64_t orc_num_roots(int32_t n_u, int32_t n_v, const int32_t *u_off, const int32_t *v_off, int side) {
    side = pick_side(n_u, n_v, side);
    const int32_t *off = side == 2 ? v_off : u_off;
    int32_t n = side == 2 ? n_v : n_u;
    int64_t k = 0;
    for (int32_t v = 0; v < n; v++) k += off[v + 1] > off[v];
    return k;
}

/*
 * The definition written out (section II-A): for every non-empty A subset of U, take
 * B = N(A) (the common neighbours of A); (A, B) is a maximal biclique exactly when B is
 * non-empty and N(B) = A.  Needs |U| <= 24 and |V| <= 64.  Records go to buf in increasing
 * order of the bitmask of A.  Returns the number of records, or -1 if the sizes are too
 * big or buf is too small.
 */
int64_t orc_brute(int32_t n_u, int32_t n_v, const int32_t *u_off, const int32_t *u_adj,
                  int32_t *buf, int64_t buf_cap, uint64_t *hash_out, int64_t *ints_out) {
    if (n_u > 24 || n_v > 64 || n_u < 0 || n_v < 0) return -1;
    uint64_t row[24];
    for (int32_t u = 0; u < n_u; u++) {
        row[u] = 0;
        for (int32_t e = u_off[u]; e < u_off[u + 1]; e++) row[u] |= 1ULL << u_adj[e];
    }
    uint64_t all_v = n_v == 64 ? ~0ULL : ((1ULL << n_v) - 1ULL);
    int64_t count = 0, w = 0;
    uint64_t hsum = 0;
    int32_t a[24], b[64];
    for (uint64_t amask = 1; amask < (1ULL << n_u); amask++) {
        uint64_t bmask = all_v;                       /* N(A) */
        for (int32_t u = 0; u < n_u; u++) if (amask >> u & 1ULL) bmask &= row[u];
        if (bmask == 0) continue;
        uint64_t nb_of_b = 0;                         /* N(B): u adjacent to all of B */
        for (int32_t u = 0; u < n_u; u++) if ((row[u] & bmask) == bmask) nb_of_b |= 1ULL << u;
        if (nb_of_b != amask) continue;
        int32_t na = 0, nb = 0;
        for (int32_t u = 0; u < n_u; u++) if (amask >> u & 1ULL) a[na++] = u;
        for (int32_t v = 0; v < n_v; v++) if (bmask >> v & 1ULL) b[nb++] = v;
        hsum += orc_hash_pair(a, na, b, nb);
        count++;
        if (buf) {
            if (w + 2 + na + nb > buf_cap) return -1;
            buf[w] = na; buf[w + 1] = nb;
            memcpy(buf + w + 2, a, sizeof(int32_t) * (size_t)na);
            memcpy(buf + w + 2 + na, b, sizeof(int32_t) * (size_t)nb);
        }
        w += 2 + na + nb;
    }
    if (hash_out) *hash_out = hsum;
    if (ints_out) *ints_out = w;
    return count;
}
