/*
 * FP64 CPU oracle for OBK-RCM (Liang & Li, "OBK-RCM: Accelerated Orthogonal
 * Block Kaczmarz Algorithm via RCM Reordering and Dynamic Grouping").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 * Every floating-point sum below runs sequentially in the stated order; every
 * + - * / sqrt is a single IEEE-754 round-to-nearest operation (no FMA
 * contraction), which is what makes bit-exact plan parity well defined.
 *
 * Readings of the paper that this file fixes (where the text is silent):
 *  - one block = one row of the reordered matrix, so a block's centroid is the
 *    row itself and the cosine table becomes exact row cosines (Section 3.3);
 *  - |cos| is compared with the threshold, a pair is near-orthogonal iff
 *    |cos| < delta (strict, as written in Section 3.3);
 *  - classes are maximal: first-fit greedy colouring in reordered row order
 *    (the pair rule of Section 3.3 is kept as orc_pairs for tests);
 *  - RCM tie-break: start at the unvisited vertex of least (degree, index),
 *    visit unvisited neighbours by ascending (degree, index), reverse the
 *    whole Cuthill-McKee sequence (Section 3.2 gives no tie-break);
 *  - one sweep projects every group once in ascending group id, all rows of a
 *    group from the same iterate (simultaneous form of eq. 3.3).
 *
 * Status: every function is pinned by the CPU test-suite (pseudo-inverse block
 * projection, sequential Kaczmarz, dense Gram cosines, hand-worked RCM orders,
 * closed forms).  The iterate after K sweeps on near-orthogonal (not exactly
 * orthogonal) groups is pinned only through convergence and non-expansiveness:
 * the paper prints no iterate values.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* Threads of the row-parallel loops (conflicts, the threaded sweep); 1
 * without OpenMP.  Only the CPU timing baseline changes it.                 */
void orc_set_threads(int t)
{
#ifdef _OPENMP
    omp_set_num_threads(t > 0 ? t : 1);
#else
    (void)t;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_CSR (-2)
#define ORC_E_NONFINITE (-4)
#define ORC_E_NOMEM (-5)

/* ---------------------------------------------------------------- O1 ----
 * Validate a square CSR (the method needs m = n, Section 4 opening).
 * Columns in range, no duplicate (row, col), values and f finite.
 * Rows need not be sorted.                                                  */
int orc_validate(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                 const double *f)
{
    if (n < 0 || !rp) return ORC_E_ARG;
    if (rp[0] != 0) return ORC_E_CSR;
    for (int64_t i = 0; i < n; i++)
        if (rp[i + 1] < rp[i]) return ORC_E_CSR;
    int64_t nnz = rp[n];
    for (int64_t k = 0; k < nnz; k++)
        if (ci[k] < 0 || (int64_t)ci[k] >= n) return ORC_E_CSR;
    /* duplicates: mark columns of each row in a scratch array */
    int64_t *seen = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!seen) return ORC_E_NOMEM;
    for (int64_t c = 0; c < n; c++) seen[c] = -1;
    int rc = ORC_OK;
    for (int64_t i = 0; i < n && rc == ORC_OK; i++)
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
            if (seen[ci[k]] == i) { rc = ORC_E_CSR; break; }
            seen[ci[k]] = i;
        }
    free(seen);
    if (rc != ORC_OK) return rc;
    for (int64_t k = 0; k < nnz; k++)
        if (!isfinite(v[k])) return ORC_E_NONFINITE;
    if (f)
        for (int64_t i = 0; i < n; i++)
            if (!isfinite(f[i])) return ORC_E_NONFINITE;
    return ORC_OK;
}

/* ---------------------------------------------------------------- O2 ----
 * Undirected simple graph of the pattern of A + A^T without the diagonal:
 * edge {u,v} iff u != v and (u,v) or (v,u) is stored.  Built as a sorted,
 * de-duplicated list of directed pairs (both directions).                   */
typedef struct { int32_t a, b; } orc_pair;

static int cmp_pair(const void *x, const void *y)
{
    const orc_pair *p = (const orc_pair *)x, *q = (const orc_pair *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return 0;
}

/* adjacency in CSR form: gp[n+1], gi[gp[n]]; returns number of entries or <0 */
static int64_t build_graph(int64_t n, const int64_t *rp, const int32_t *ci,
                           int64_t **gp_out, int32_t **gi_out)
{
    int64_t nnz = rp[n];
    orc_pair *e = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(2 * nnz + 1));
    if (!e) return ORC_E_NOMEM;
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
            int32_t j = ci[k];
            if (j == (int32_t)i) continue;
            e[m].a = (int32_t)i; e[m].b = j; m++;
            e[m].a = j; e[m].b = (int32_t)i; m++;
        }
    qsort(e, (size_t)m, sizeof(orc_pair), cmp_pair);
    int64_t u = 0;
    for (int64_t t = 0; t < m; t++)
        if (t == 0 || cmp_pair(&e[t], &e[t - 1]) != 0) e[u++] = e[t];
    int64_t *gp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *gi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(u + 1));
    if (!gp || !gi) { free(e); free(gp); free(gi); return ORC_E_NOMEM; }
    for (int64_t t = 0; t < u; t++) gp[e[t].a + 1]++;
    for (int64_t i = 0; i < n; i++) gp[i + 1] += gp[i];
    for (int64_t t = 0; t < u; t++) gi[t] = e[t].b;   /* already grouped by a */
    free(e);
    *gp_out = gp; *gi_out = gi;
    return u;
}

/* ---------------------------------------------------------------- O3 ----
 * Reverse Cuthill-McKee (Section 3.2; Algorithm 4, first step).
 * Cuthill-McKee: while a vertex is unvisited, start a breadth-first search at
 * the unvisited vertex of least (degree, index); a dequeued vertex is appended
 * to the order and its unvisited neighbours, sorted by (degree, index), are
 * marked visited and enqueued.  The concatenated order is then reversed.
 * Output p[t] = old index of new row t (new -> old).                        */
static const int64_t *g_deg_for_sort;
static int cmp_deg_idx(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    int64_t da = g_deg_for_sort[a], db = g_deg_for_sort[b];
    if (da != db) return da < db ? -1 : 1;
    return (a > b) - (a < b);
}

int orc_rcm(int64_t n, const int64_t *rp, const int32_t *ci, int32_t *p)
{
    if (n == 0) return ORC_OK;
    int64_t *gp; int32_t *gi;
    int64_t ne = build_graph(n, rp, ci, &gp, &gi);
    if (ne < 0) return (int)ne;
    int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *byrank = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    char *visited = (char *)calloc((size_t)n, 1);
    if (!deg || !byrank || !queue || !order || !nb || !visited) {
        free(gp); free(gi); free(deg); free(byrank); free(queue); free(order); free(nb); free(visited);
        return ORC_E_NOMEM;
    }
    for (int64_t v = 0; v < n; v++) { deg[v] = gp[v + 1] - gp[v]; byrank[v] = (int32_t)v; }
    /* all vertices sorted by (degree, index): the first unvisited entry of this
     * list is the argmin over unvisited vertices */
    g_deg_for_sort = deg;
    qsort(byrank, (size_t)n, sizeof(int32_t), cmp_deg_idx);
    int64_t cursor = 0, norder = 0;
    while (norder < n) {
        while (visited[byrank[cursor]]) cursor++;
        int32_t s = byrank[cursor];
        int64_t head = 0, tail = 0;
        visited[s] = 1;
        queue[tail++] = s;
        while (head < tail) {
            int32_t v = queue[head++];
            order[norder++] = v;
            int64_t cnt = 0;
            for (int64_t k = gp[v]; k < gp[v + 1]; k++)
                if (!visited[gi[k]]) nb[cnt++] = gi[k];
            qsort(nb, (size_t)cnt, sizeof(int32_t), cmp_deg_idx);
            for (int64_t t = 0; t < cnt; t++) { visited[nb[t]] = 1; queue[tail++] = nb[t]; }
        }
    }
    for (int64_t t = 0; t < n; t++) p[t] = order[n - 1 - t];
    free(gp); free(gi); free(deg); free(byrank); free(queue); free(order); free(nb); free(visited);
    return ORC_OK;
}

/* ---------------------------------------------------------------- O4 ----
 * Symmetric permutation, eqs. (3.1)-(3.2): row t of A~ = P A P^T is row p[t]
 * of A with every column c renamed q[c] (q = inverse of p) and the row sorted
 * ascending by the new column; f~_t = f_{p[t]}.                              */
typedef struct { int32_t c; double v; } orc_entry;
static int cmp_entry(const void *x, const void *y)
{
    int32_t a = ((const orc_entry *)x)->c, b = ((const orc_entry *)y)->c;
    return (a > b) - (a < b);
}

int orc_permute(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                const double *f, const int32_t *p, int64_t *trp, int32_t *tci, double *tv,
                double *tf)
{
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    orc_entry *buf = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)(n > 0 ? n : 1));
    if (!q || !buf) { free(q); free(buf); return ORC_E_NOMEM; }
    for (int64_t t = 0; t < n; t++) q[p[t]] = (int32_t)t;
    trp[0] = 0;
    for (int64_t t = 0; t < n; t++) {
        int32_t old = p[t];
        int64_t len = rp[old + 1] - rp[old];
        for (int64_t k = 0; k < len; k++) {
            buf[k].c = q[ci[rp[old] + k]];
            buf[k].v = v[rp[old] + k];
        }
        qsort(buf, (size_t)len, sizeof(orc_entry), cmp_entry);
        for (int64_t k = 0; k < len; k++) {
            tci[trp[t] + k] = buf[k].c;
            tv[trp[t] + k] = buf[k].v;
        }
        trp[t + 1] = trp[t] + len;
        if (tf && f) tf[t] = f[old];
    }
    free(q); free(buf);
    return ORC_OK;
}

/* ---------------------------------------------------------------- O5 ----
 * Squared row norms, the denominator of eq. (1.2): nu_i = sum_k a_ik^2 in
 * ascending k; inv_i = 1/nu_i (0 for an all-zero row, which is never
 * projected).                                                               */
void orc_norms(int64_t n, const int64_t *rp, const double *v, double *nu, double *inv)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * v[k];
        nu[i] = s;
        inv[i] = (s != 0.0) ? 1.0 / s : 0.0;
    }
}

/* ---------------------------------------------------------------- O6 ----
 * Row cosines (the cosine table C of Section 3.3 with one-row blocks).
 * For rows i, j sharing at least one column: d = sum over the common columns
 * in ascending order of a_ic * a_jc; cos_ij = |d| / sqrt(nu_i * nu_j)
 * (product rounded, then sqrt, then the division).  Rows sharing no column are
 * exactly orthogonal.  The pair conflicts (is NOT near-orthogonal) iff
 * cos_ij >= delta.  Zero rows take part in nothing.
 * Rows must be sorted ascending (O4 output).
 *
 * Output, for each i, the conflicting j < i in ascending order:
 *   cptr[n+1], cidx[cptr[n]].  With cidx == NULL only cptr is filled.       */
static double sparse_dot_sorted(const int32_t *ca, const double *va, int64_t la,
                                const int32_t *cb, const double *vb, int64_t lb, int *shared)
{
    double d = 0.0;
    int64_t a = 0, b = 0;
    *shared = 0;
    while (a < la && b < lb) {
        if (ca[a] < cb[b]) a++;
        else if (ca[a] > cb[b]) b++;
        else { d = d + va[a] * vb[b]; *shared = 1; a++; b++; }
    }
    return d;
}

double orc_cosine(int64_t i, int64_t j, const int64_t *rp, const int32_t *ci, const double *v,
                  const double *nu)
{
    int shared;
    double d = sparse_dot_sorted(ci + rp[i], v + rp[i], rp[i + 1] - rp[i],
                                 ci + rp[j], v + rp[j], rp[j + 1] - rp[j], &shared);
    if (!shared || nu[i] == 0.0 || nu[j] == 0.0) return 0.0;
    return fabs(d) / sqrt(nu[i] * nu[j]);
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* The conflicts of one row i: the rows j < i sharing a column with it, in
 * ascending order, whose cosine reaches delta.  Writes them to out (may be
 * NULL) and returns their count.  mark[] / cand[] are scratch of n entries
 * (mark[j] != i on entry for every j).                                      */
static int64_t row_conflicts(int64_t i, const int64_t *rp, const int32_t *ci, const double *v,
                             const double *nu, double delta, const int64_t *cp, const int32_t *cr,
                             int64_t *mark, int32_t *cand, int32_t *out)
{
    int64_t ncand = 0, cnt = 0;
    if (nu[i] == 0.0) return 0;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
        int32_t c = ci[k];
        for (int64_t t = cp[c]; t < cp[c + 1]; t++) {
            int32_t j = cr[t];
            if (j < i && mark[j] != i) { mark[j] = i; cand[ncand++] = j; }
        }
    }
    qsort(cand, (size_t)ncand, sizeof(int32_t), cmp_i32);
    for (int64_t t = 0; t < ncand; t++) {
        int32_t j = cand[t];
        if (nu[j] == 0.0) continue;
        if (orc_cosine(i, j, rp, ci, v, nu) >= delta) {
            if (out) out[cnt] = j;
            cnt++;
        }
    }
    return cnt;
}

/* Rows are independent, so the count and fill passes may run on several
 * threads (OpenMP when built with it); each row's list is the same.          */
int64_t orc_conflicts(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                      const double *nu, double delta, int64_t *cptr, int32_t *cidx)
{
    /* column -> rows (CSC of the pattern) */
    int64_t nnz = rp[n];
    int64_t *cp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *cr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!cp || !cr || !fill) { free(cp); free(cr); free(fill); return ORC_E_NOMEM; }
    for (int64_t k = 0; k < nnz; k++) cp[ci[k] + 1]++;
    for (int64_t c = 0; c < n; c++) cp[c + 1] += cp[c];
    for (int64_t c = 0; c < n; c++) fill[c] = cp[c];
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) cr[fill[ci[k]]++] = (int32_t)i;

    /* counts per row (cptr[i + 1]), then offsets; with cidx, the lists */
    int failed = 0;
    for (int pass = 0; pass < (cidx ? 2 : 1); pass++) {
        #pragma omp parallel
        {
            int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
            int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
            if (!mark || !cand) {
                #pragma omp atomic write
                failed = 1;
            } else {
                for (int64_t j = 0; j < n; j++) mark[j] = -1;
                #pragma omp for schedule(dynamic, 1024)
                for (int64_t i = 0; i < n; i++) {
                    if (pass == 0) cptr[i + 1] = row_conflicts(i, rp, ci, v, nu, delta, cp, cr, mark, cand, NULL);
                    else (void)row_conflicts(i, rp, ci, v, nu, delta, cp, cr, mark, cand, cidx + cptr[i]);
                }
            }
            free(mark);
            free(cand);
        }
        if (failed) break;
        if (pass == 0) {
            cptr[0] = 0;
            for (int64_t i = 0; i < n; i++) cptr[i + 1] += cptr[i];
        }
    }
    free(cp); free(cr); free(fill);
    return failed ? ORC_E_NOMEM : cptr[n];
}

/* ---------------------------------------------------------------- O7 ----
 * Grouping (Section 3.3, class{i}, Oclass/Nclass; Algorithm 4, fourth step).
 * Taking "the first later block orthogonal to A_i" to its maximal form: rows
 * are visited in reordered order and row i joins the lowest-numbered group
 * that holds no row conflicting with it (first-fit greedy colouring of the
 * conflict graph).  A zero row joins no group (group -1).
 * Returns the number of groups.                                             */
int32_t orc_groups(int64_t n, const double *nu, const int64_t *cptr, const int32_t *cidx,
                   int32_t *group)
{
    char *used = (char *)calloc((size_t)n + 2, 1);
    if (!used) return ORC_E_NOMEM;
    int32_t ngroups = 0;
    for (int64_t i = 0; i < n; i++) {
        if (nu[i] == 0.0) { group[i] = -1; continue; }
        for (int64_t t = cptr[i]; t < cptr[i + 1]; t++)
            if (group[cidx[t]] >= 0) used[group[cidx[t]]] = 1;
        int32_t g = 0;
        while (used[g]) g++;
        group[i] = g;
        if (g + 1 > ngroups) ngroups = g + 1;
        for (int64_t t = cptr[i]; t < cptr[i + 1]; t++)
            if (group[cidx[t]] >= 0) used[group[cidx[t]]] = 0;
    }
    free(used);
    return ngroups;
}

/* The literal pair rule of Section 3.3: for each unassigned row i (ascending),
 * the first unassigned later row j with cos_ij < delta forms class{i} = {i, j};
 * a row that finds no partner goes to Nclass.  Output: pair_of[i] = partner
 * (or -1 for an Nclass row, -2 for a zero row).  Quadratic; tiny inputs.     */
int orc_pairs(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
              const double *nu, double delta, int32_t *pair_of)
{
    for (int64_t i = 0; i < n; i++) pair_of[i] = (nu[i] == 0.0) ? -2 : -3;   /* -3: unassigned */
    for (int64_t i = 0; i < n; i++) {
        if (pair_of[i] != -3) continue;
        pair_of[i] = -1;
        for (int64_t j = i + 1; j < n; j++) {
            if (pair_of[j] != -3) continue;
            if (orc_cosine(i, j, rp, ci, v, nu) < delta) {
                pair_of[i] = (int32_t)j; pair_of[j] = (int32_t)i; break;
            }
        }
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- O8 ----
 * One OBK sweep (eq. 3.3 with one-row blocks; eq. 1.2 per row).
 * For g = 0 .. ngroups-1:
 *   (i)  for every row i of group g, from the same iterate x:
 *          s = sum_k a_ik x_k (ascending k);  w_i = ((f_i - s) * inv_i) * omega
 *   (ii) for every column c touched by group g:
 *          t = sum over rows i of group g holding c, ascending i, of w_i a_ic;
 *          x_c = x_c + t
 * For exactly orthogonal rows this is the pseudo-inverse projection of eq.
 * (1.3); for near-orthogonal rows it defines the step.  `sweeps` sweeps run.
 * omega is a relaxation of every row step; the paper's step is omega = 1
 * (multiplying by 1.0 is exact, so that case is the unrelaxed step bit for
 * bit).  T = double (FP64).                                                  */
int orc_sweep(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
              const double *f, const double *inv, const int32_t *group, int32_t ngroups,
              double omega, double *x, int64_t sweeps)
{
    /* rows of each group in ascending order */
    int64_t *gp = (int64_t *)calloc((size_t)ngroups + 1, sizeof(int64_t));
    int32_t *gr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ngroups + 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *t = (double *)calloc((size_t)n + 1, sizeof(double));
    char *touched = (char *)calloc((size_t)n + 1, 1);
    int32_t *tlist = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!gp || !gr || !fill || !w || !t || !touched || !tlist) {
        free(gp); free(gr); free(fill); free(w); free(t); free(touched); free(tlist);
        return ORC_E_NOMEM;
    }
    for (int64_t i = 0; i < n; i++) if (group[i] >= 0) gp[group[i] + 1]++;
    for (int32_t g = 0; g < ngroups; g++) gp[g + 1] += gp[g];
    for (int32_t g = 0; g < ngroups; g++) fill[g] = gp[g];
    for (int64_t i = 0; i < n; i++) if (group[i] >= 0) gr[fill[group[i]]++] = (int32_t)i;

    for (int64_t it = 0; it < sweeps; it++) {
        for (int32_t g = 0; g < ngroups; g++) {
            /* (i) residual weights from the same iterate */
            for (int64_t a = gp[g]; a < gp[g + 1]; a++) {
                int32_t i = gr[a];
                double s = 0.0;
                for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * x[ci[k]];
                w[i] = ((f[i] - s) * inv[i]) * omega;
            }
            /* (ii) per touched column, the sum over the group's rows in
             * ascending row order, then one update of x_c */
            int64_t nt = 0;
            for (int64_t a = gp[g]; a < gp[g + 1]; a++) {
                int32_t i = gr[a];
                for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
                    int32_t c = ci[k];
                    if (!touched[c]) { touched[c] = 1; t[c] = 0.0; tlist[nt++] = c; }
                    t[c] = t[c] + w[i] * v[k];
                }
            }
            for (int64_t a = 0; a < nt; a++) {
                int32_t c = tlist[a];
                x[c] = x[c] + t[c];
                touched[c] = 0;
            }
        }
    }
    free(gp); free(gr); free(fill); free(w); free(t); free(touched); free(tlist);
    return ORC_OK;
}

/* The same sweep on several threads (OpenMP), for the CPU timing baseline
 * and the full-size checks: phase (i) over the rows of a group, phase (ii)
 * over the columns it touches, each column summing its group's entries in
 * ascending row order before the one update of x_c -- the arithmetic of
 * orc_sweep, operation for operation, so the iterates are equal bit for bit.
 * orc_mt_prepare lays out, per group, the touched columns and their entries
 * (row, value) by ascending row; orc_mt_sweep runs sweeps; orc_mt_free.    */
typedef struct {
    int64_t n;
    int32_t ngroups;
    int64_t *gp;       /* rows of group g: gr[gp[g] .. gp[g+1]) */
    int32_t *gr;
    int64_t *tp;       /* touched columns of group g: tc[tp[g] .. tp[g+1]) */
    int32_t *tc;
    int64_t *ep;       /* entries of touched column t: [ep[t], ep[t+1]) */
    int32_t *er;       /* row of each entry */
    double *ev;        /* value of each entry */
    double *w;
} orc_mt;

void orc_mt_free(orc_mt *h)
{
    if (!h) return;
    free(h->gp); free(h->gr); free(h->tp); free(h->tc); free(h->ep); free(h->er); free(h->ev); free(h->w);
    free(h);
}

orc_mt *orc_mt_prepare(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                       const int32_t *group, int32_t ngroups)
{
    orc_mt *h = (orc_mt *)calloc(1, sizeof(orc_mt));
    if (!h) return NULL;
    int64_t nnz = rp[n];
    h->n = n;
    h->ngroups = ngroups;
    h->gp = (int64_t *)calloc((size_t)ngroups + 1, sizeof(int64_t));
    h->gr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    h->tp = (int64_t *)calloc((size_t)ngroups + 1, sizeof(int64_t));
    h->tc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    h->ep = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz + 2));
    h->er = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    h->ev = (double *)malloc(sizeof(double) * (size_t)(nnz + 1));
    h->w = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *slot = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!h->gp || !h->gr || !h->tp || !h->tc || !h->ep || !h->er || !h->ev || !h->w || !cnt || !slot) {
        free(cnt); free(slot); orc_mt_free(h); return NULL;
    }
    for (int64_t i = 0; i < n; i++) if (group[i] >= 0) h->gp[group[i] + 1]++;
    for (int32_t g = 0; g < ngroups; g++) h->gp[g + 1] += h->gp[g];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ngroups + 1));
        if (!fill) { free(cnt); free(slot); orc_mt_free(h); return NULL; }
        for (int32_t g = 0; g < ngroups; g++) fill[g] = h->gp[g];
        for (int64_t i = 0; i < n; i++) if (group[i] >= 0) h->gr[fill[group[i]]++] = (int32_t)i;
        free(fill);
    }
    /* per group: entries counted per column, touched columns ascending,
     * then filled by ascending row */
    int64_t nt = 0, ne = 0;
    for (int32_t g = 0; g < ngroups; g++) {
        h->tp[g] = nt;
        for (int64_t a = h->gp[g]; a < h->gp[g + 1]; a++) {
            int32_t i = h->gr[a];
            for (int64_t k = rp[i]; k < rp[i + 1]; k++) cnt[ci[k]]++;
        }
        int64_t t0 = nt;
        for (int64_t a = h->gp[g]; a < h->gp[g + 1]; a++) {
            int32_t i = h->gr[a];
            for (int64_t k = rp[i]; k < rp[i + 1]; k++)
                if (cnt[ci[k]] > 0 && slot[ci[k]] != -1 - (int64_t)g) {
                    slot[ci[k]] = -1 - (int64_t)g;
                    h->tc[nt++] = ci[k];
                }
        }
        qsort(h->tc + t0, (size_t)(nt - t0), sizeof(int32_t), cmp_i32);
        for (int64_t t = t0; t < nt; t++) {
            int32_t c = h->tc[t];
            h->ep[t] = ne;
            slot[c] = ne;
            ne += cnt[c];
            cnt[c] = 0;
        }
        for (int64_t a = h->gp[g]; a < h->gp[g + 1]; a++) {
            int32_t i = h->gr[a];
            for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
                int64_t e = slot[ci[k]]++;
                h->er[e] = i;
                h->ev[e] = v[k];
            }
        }
        for (int64_t t = t0; t < nt; t++) slot[h->tc[t]] = 0;
    }
    h->tp[ngroups] = nt;
    h->ep[nt] = ne;
    free(cnt); free(slot);
    return h;
}

int orc_mt_sweep(const orc_mt *h, const int64_t *rp, const int32_t *ci, const double *v,
                 const double *f, const double *inv, double omega, double *x, int64_t sweeps)
{
    if (!h) return ORC_E_ARG;
    double *w = h->w;
    for (int64_t it = 0; it < sweeps; it++) {
        for (int32_t g = 0; g < h->ngroups; g++) {
            #pragma omp parallel for schedule(static)
            for (int64_t a = h->gp[g]; a < h->gp[g + 1]; a++) {
                int32_t i = h->gr[a];
                double s = 0.0;
                for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * x[ci[k]];
                w[i] = ((f[i] - s) * inv[i]) * omega;
            }
            #pragma omp parallel for schedule(static)
            for (int64_t t = h->tp[g]; t < h->tp[g + 1]; t++) {
                double tt = 0.0;
                for (int64_t e = h->ep[t]; e < h->ep[t + 1]; e++) tt = tt + w[h->er[e]] * h->ev[e];
                x[h->tc[t]] = x[h->tc[t]] + tt;
            }
        }
    }
    return ORC_OK;
}

/* Sequential row projections in a given row order (eq. 1.2 applied row by
 * row, each from the latest iterate).  Used to pin O8 (P3) and the pair mode
 * of Algorithm 4, where the two blocks of a class are projected one after the
 * other.                                                                     */
void orc_rowwise(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                 const double *f, const double *inv, const int32_t *rows, int64_t nrows,
                 double *x)
{
    (void)n;
    for (int64_t a = 0; a < nrows; a++) {
        int32_t i = rows[a];
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * x[ci[k]];
        double w = (f[i] - s) * inv[i];
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) x[ci[k]] = x[ci[k]] + w * v[k];
    }
}

/* ---------------------------------------------------------------- O9 ----
 * Residual r = f - A x (ascending k per row) and the relative residual
 * ||r||_2 / ||f||_2, each norm the sqrt of an ascending-index sum of squares.
 * r may be NULL.  Returns -1 if ||f|| = 0 and ||r|| > 0, 0 if both are 0.     */
double orc_relres(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                  const double *f, const double *x, double *r)
{
    double rr = 0.0, ff = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * x[ci[k]];
        double ri = f[i] - s;
        if (r) r[i] = ri;
        rr = rr + ri * ri;
        ff = ff + f[i] * f[i];
    }
    if (ff == 0.0) return rr == 0.0 ? 0.0 : -1.0;
    return sqrt(rr) / sqrt(ff);
}

/* --------------------------------------------------------------- O10 ----
 * Back-permutation x = P^T x~ (Algorithm 4, last step): x[p[t]] = xt[t].    */
void orc_unpermute(int64_t n, const int32_t *p, const double *xt, double *x)
{
    for (int64_t t = 0; t < n; t++) x[p[t]] = xt[t];
}

/* Forward permutation of a vector: xt[t] = x[p[t]].                          */
void orc_permute_vec(int64_t n, const int32_t *p, const double *x, double *xt)
{
    for (int64_t t = 0; t < n; t++) xt[t] = x[p[t]];
}

/* --------------------------------------------------------------- O11 ----
 * Iterative refinement around the sweep (not in the paper): with x~ in FP64,
 *   r = f - A x;  stop if ||r||/||f|| <= tol or `outer` steps are done;
 *   sigma = max_i |r_i|;  b = r / sigma;
 *   d = 0;  `inner` sweeps of O8 on A d = b (same groups and order);
 *   x = x + sigma * d.
 * The oracle runs this schedule in FP64 throughout, so a GPU run of the same
 * schedule with an FP32 inner sweep differs only by the FP32 inner arithmetic.
 * Returns the number of outer steps taken; *relres gets the last residual.  */
int64_t orc_refine(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                   const double *f, const double *inv, const int32_t *group, int32_t ngroups,
                   double omega, double *x, int64_t inner, int64_t outer, double tol, double *relres)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *d = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!r || !d) { free(r); free(d); return ORC_E_NOMEM; }
    int64_t steps = 0;
    double rho = orc_relres(n, rp, ci, v, f, x, r);
    while (!(rho <= tol) && steps < outer) {
        double sigma = 0.0;
        for (int64_t i = 0; i < n; i++) if (fabs(r[i]) > sigma) sigma = fabs(r[i]);
        if (sigma == 0.0) break;
        for (int64_t i = 0; i < n; i++) { r[i] = r[i] / sigma; d[i] = 0.0; }
        orc_sweep(n, rp, ci, v, r, inv, group, ngroups, omega, d, inner);
        for (int64_t i = 0; i < n; i++) x[i] = x[i] + sigma * d[i];
        steps++;
        rho = orc_relres(n, rp, ci, v, f, x, r);
    }
    if (relres) *relres = rho;
    free(r); free(d);
    return steps;
}

/* --------------------------------------------------------------- O9 -----
 * Solve to a tolerance (the stopping rule of Section 3.5, read as a relative
 * residual): from x (x~0 on entry, the iterate on return)
 *   rho0 = ||f - A x|| / ||f||;
 *   NONFINITE if some residual entry or the sum of squares is not finite,
 *   else CONVERGED at once if tol > 0 and rho0 <= tol;
 *   while fewer than maxit sweeps are done and no outcome is set:
 *     run c = min(check_every, maxit - done) sweeps (all maxit - done when
 *     tol <= 0), then, if tol > 0, recompute rho:
 *       NONFINITE as above, else CONVERGED if rho <= tol, else DIVERGED if
 *       rho0 > 0 and rho > 1e3 rho0;
 *   with tol <= 0, rho is computed once after the maxit sweeps.
 * "Not finite" is read from the residual's sum of squares (a NaN or infinite
 * entry makes it so).  Each norm is the sqrt of an ascending-index sum of
 * squares; ||f|| = 0
 * gives rho = 0 when ||r|| = 0 and +inf otherwise.  out[0] = sweeps done,
 * out[1] = residual checks after sweeps; rho[0] = rho0, rho[1] = last rho.
 * Returns the outcome (ORC_CONVERGED ... ORC_NONFINITE) or an error < 0.    */
#define ORC_CONVERGED 0
#define ORC_MAXIT 1
#define ORC_DIVERGED 2
#define ORC_NONFINITE 3

static double relres_flag(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                          const double *f, const double *x, int *nonfinite)
{
    double rr = 0.0, ff = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * x[ci[k]];
        double ri = f[i] - s;
        rr = rr + ri * ri;
        ff = ff + f[i] * f[i];
    }
    /* a NaN or infinite residual entry makes the sum NaN or infinite */
    *nonfinite = !isfinite(rr);
    if (ff == 0.0) return rr == 0.0 ? 0.0 : INFINITY;
    return sqrt(rr) / sqrt(ff);
}

int orc_solve_tol(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                  const double *f, const double *inv, const int32_t *group, int32_t ngroups,
                  double omega, double *x, double tol, int64_t maxit, int64_t check_every, int64_t *out,
                  double *rho)
{
    if (n < 0 || maxit < 0 || check_every < 1 || !out || !rho) return ORC_E_ARG;
    int bad = 0;
    double rho0 = relres_flag(n, rp, ci, v, f, x, &bad);
    double cur = rho0;
    int status = ORC_MAXIT;
    int64_t done = 0, checks = 0;
    if (bad) status = ORC_NONFINITE;
    else if (tol > 0.0 && rho0 <= tol) status = ORC_CONVERGED;
    while (done < maxit && status == ORC_MAXIT) {
        int64_t c = maxit - done;
        if (tol > 0.0 && check_every < c) c = check_every;
        int rc = orc_sweep(n, rp, ci, v, f, inv, group, ngroups, omega, x, c);
        if (rc != ORC_OK) return rc;
        done += c;
        if (tol > 0.0) {
            checks++;
            cur = relres_flag(n, rp, ci, v, f, x, &bad);
            if (bad) status = ORC_NONFINITE;
            else if (cur <= tol) status = ORC_CONVERGED;
            else if (rho0 > 0.0 && cur > 1e3 * rho0) status = ORC_DIVERGED;
        }
    }
    if (tol <= 0.0) cur = relres_flag(n, rp, ci, v, f, x, &bad);
    out[0] = done;
    out[1] = checks;
    rho[0] = rho0;
    rho[1] = cur;
    return status;
}

/* ------------------------------------------------------------- complex ----
 * The complex case: the paper solves the complex matrix kim1 with the same
 * algorithm (its discussion of Table 4).  Entries are held as separate real
 * (vr) and imaginary (vi) arrays on the pattern of O4.  Over C:
 *   row norm        nu_i = sum_k (re a_ik^2 + im a_ik^2), ascending k;
 *   row cosine      d = a_i^H a_j = sum over common columns, ascending, of
 *                   conj(a_ic) a_jc, i.e. with a = a_ic, b = a_jc:
 *                     re d = re d + (re a re b + im a im b),
 *                     im d = im d + (re a im b - im a re b);
 *                   cos_ij = sqrt(re d^2 + im d^2) / sqrt(nu_i nu_j);
 *   row projection  eq. (1.2) over C: x = x + (f_i - a_i x) / nu_i a_i^H, with
 *                     a_i x = sum_k a_ik x_k (ascending k),
 *                     re += re a re x - im a im x, im += re a im x + im a re x,
 *                   and the update of x_c adding w conj(a_ic):
 *                     re += re w re a + im w im a, im += im w re a - re w im a.
 * The group sweep is O8 with these operations; each sum is accumulated in
 * the order given.                                                          */
void orc_norms_z(int64_t n, const int64_t *rp, const double *vr, const double *vi, double *nu, double *inv)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + (vr[k] * vr[k] + vi[k] * vi[k]);
        nu[i] = s;
        inv[i] = (s != 0.0) ? 1.0 / s : 0.0;
    }
}

double orc_cosine_z(int64_t i, int64_t j, const int64_t *rp, const int32_t *ci, const double *vr,
                    const double *vi, const double *nu)
{
    double dr = 0.0, di = 0.0;
    int shared = 0;
    int64_t a = rp[i], b = rp[j];
    while (a < rp[i + 1] && b < rp[j + 1]) {
        if (ci[a] < ci[b]) a++;
        else if (ci[a] > ci[b]) b++;
        else {
            dr = dr + (vr[a] * vr[b] + vi[a] * vi[b]);
            di = di + (vr[a] * vi[b] - vi[a] * vr[b]);
            shared = 1;
            a++;
            b++;
        }
    }
    if (!shared || nu[i] == 0.0 || nu[j] == 0.0) return 0.0;
    return sqrt(dr * dr + di * di) / sqrt(nu[i] * nu[j]);
}

int64_t orc_conflicts_z(int64_t n, const int64_t *rp, const int32_t *ci, const double *vr, const double *vi,
                        const double *nu, double delta, int64_t *cptr, int32_t *cidx)
{
    int64_t nnz = rp[n];
    int64_t *cp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *cr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!cp || !cr || !fill || !mark || !cand) {
        free(cp); free(cr); free(fill); free(mark); free(cand); return ORC_E_NOMEM;
    }
    for (int64_t k = 0; k < nnz; k++) cp[ci[k] + 1]++;
    for (int64_t c = 0; c < n; c++) cp[c + 1] += cp[c];
    for (int64_t c = 0; c < n; c++) fill[c] = cp[c];
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) cr[fill[ci[k]]++] = (int32_t)i;
    for (int64_t j = 0; j < n; j++) mark[j] = -1;
    int64_t total = 0;
    cptr[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t ncand = 0;
        if (nu[i] != 0.0) {
            for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
                int32_t c = ci[k];
                for (int64_t t = cp[c]; t < cp[c + 1]; t++) {
                    int32_t j = cr[t];
                    if (j < i && mark[j] != i) { mark[j] = i; cand[ncand++] = j; }
                }
            }
        }
        qsort(cand, (size_t)ncand, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < ncand; t++) {
            int32_t j = cand[t];
            if (nu[j] == 0.0) continue;
            if (orc_cosine_z(i, j, rp, ci, vr, vi, nu) >= delta) {
                if (cidx) cidx[total] = j;
                total++;
            }
        }
        cptr[i + 1] = total;
    }
    free(cp); free(cr); free(fill); free(mark); free(cand);
    return total;
}

int orc_sweep_z(int64_t n, const int64_t *rp, const int32_t *ci, const double *vr, const double *vi,
                const double *fr, const double *fi, const double *inv, const int32_t *group, int32_t ngroups,
                double omega, double *xr, double *xi, int64_t sweeps)
{
    int64_t *gp = (int64_t *)calloc((size_t)ngroups + 1, sizeof(int64_t));
    int32_t *gr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ngroups + 1));
    double *wr = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *wi = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *tr = (double *)calloc((size_t)n + 1, sizeof(double));
    double *ti = (double *)calloc((size_t)n + 1, sizeof(double));
    char *touched = (char *)calloc((size_t)n + 1, 1);
    int32_t *tlist = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!gp || !gr || !fill || !wr || !wi || !tr || !ti || !touched || !tlist) {
        free(gp); free(gr); free(fill); free(wr); free(wi); free(tr); free(ti); free(touched); free(tlist);
        return ORC_E_NOMEM;
    }
    for (int64_t i = 0; i < n; i++) if (group[i] >= 0) gp[group[i] + 1]++;
    for (int32_t g = 0; g < ngroups; g++) gp[g + 1] += gp[g];
    for (int32_t g = 0; g < ngroups; g++) fill[g] = gp[g];
    for (int64_t i = 0; i < n; i++) if (group[i] >= 0) gr[fill[group[i]]++] = (int32_t)i;
    for (int64_t it = 0; it < sweeps; it++) {
        for (int32_t g = 0; g < ngroups; g++) {
            for (int64_t a = gp[g]; a < gp[g + 1]; a++) {
                int32_t i = gr[a];
                double sr = 0.0, si = 0.0;
                for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
                    int32_t c = ci[k];
                    sr = sr + (vr[k] * xr[c] - vi[k] * xi[c]);
                    si = si + (vr[k] * xi[c] + vi[k] * xr[c]);
                }
                wr[i] = ((fr[i] - sr) * inv[i]) * omega;
                wi[i] = ((fi[i] - si) * inv[i]) * omega;
            }
            int64_t nt = 0;
            for (int64_t a = gp[g]; a < gp[g + 1]; a++) {
                int32_t i = gr[a];
                for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
                    int32_t c = ci[k];
                    if (!touched[c]) { touched[c] = 1; tr[c] = 0.0; ti[c] = 0.0; tlist[nt++] = c; }
                    tr[c] = tr[c] + (wr[i] * vr[k] + wi[i] * vi[k]);
                    ti[c] = ti[c] + (wi[i] * vr[k] - wr[i] * vi[k]);
                }
            }
            for (int64_t a = 0; a < nt; a++) {
                int32_t c = tlist[a];
                xr[c] = xr[c] + tr[c];
                xi[c] = xi[c] + ti[c];
                touched[c] = 0;
            }
        }
    }
    free(gp); free(gr); free(fill); free(wr); free(wi); free(tr); free(ti); free(touched); free(tlist);
    return ORC_OK;
}

/* Sequential complex row projections in a given order (eq. 1.2 over C). */
void orc_rowwise_z(int64_t n, const int64_t *rp, const int32_t *ci, const double *vr, const double *vi,
                   const double *fr, const double *fi, const double *inv, const int32_t *rows, int64_t nrows,
                   double *xr, double *xi)
{
    (void)n;
    for (int64_t a = 0; a < nrows; a++) {
        int32_t i = rows[a];
        double sr = 0.0, si = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
            int32_t c = ci[k];
            sr = sr + (vr[k] * xr[c] - vi[k] * xi[c]);
            si = si + (vr[k] * xi[c] + vi[k] * xr[c]);
        }
        double wr = (fr[i] - sr) * inv[i], wi = (fi[i] - si) * inv[i];
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
            int32_t c = ci[k];
            xr[c] = xr[c] + (wr * vr[k] + wi * vi[k]);
            xi[c] = xi[c] + (wi * vr[k] - wr * vi[k]);
        }
    }
}

/* Complex residual norm ratio ||f - A x|| / ||f|| (sums of |.|^2, ascending). */
double orc_relres_z(int64_t n, const int64_t *rp, const int32_t *ci, const double *vr, const double *vi,
                    const double *fr, const double *fi, const double *xr, const double *xi)
{
    double res2 = 0.0, rhs2 = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double sr = 0.0, si = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
            int32_t c = ci[k];
            sr = sr + (vr[k] * xr[c] - vi[k] * xi[c]);
            si = si + (vr[k] * xi[c] + vi[k] * xr[c]);
        }
        double er = fr[i] - sr, ei = fi[i] - si;
        res2 = res2 + (er * er + ei * ei);
        rhs2 = rhs2 + (fr[i] * fr[i] + fi[i] * fi[i]);
    }
    if (rhs2 == 0.0) return res2 == 0.0 ? 0.0 : -1.0;
    return sqrt(res2) / sqrt(rhs2);
}
