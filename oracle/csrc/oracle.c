/*
 * oracle.c -- plain FP64 CPU reference for the sparse LDL' factorization of
 * the KKT matrix (paper Sec. 2.2, eq. 2) and for its symbolic analysis.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU baseline of
 * the benchmark load it.  It shares no code with the device path.
 *
 * The paper only states that the analysis phase computes a fill-reducing
 * reordering and a symbolic factorization once, and that the factor phase
 * computes LDL' once per interior-point iteration (Sec. 2.2).  The ordering
 * used here is our own fully specified minimum-degree rule, written out in
 * or_min_degree below; the device library implements the same rule
 * independently and must produce the same integers.
 *
 * Everything is deliberately simple: dynamic arrays, linear scans, sorting
 * with qsort, scalar loops.  Speed is not a goal.
 */
#define _POSIX_C_SOURCE 200809L  /* clock_gettime */
#include <stdint.h>
#include <stdlib.h>
#include <time.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------ */
/* small dynamic int array                                             */
/* ------------------------------------------------------------------ */
typedef struct { int32_t *a; int32_t n, cap; } ivec;

static int iv_push(ivec *v, int32_t x) {
    if (v->n == v->cap) {
        int32_t nc = v->cap ? 2 * v->cap : 4;
        int32_t *na = (int32_t *)realloc(v->a, (size_t)nc * sizeof(int32_t));
        if (!na) return -1;
        v->a = na; v->cap = nc;
    }
    v->a[v->n++] = x;
    return 0;
}
static void iv_free(ivec *v) { free(v->a); v->a = NULL; v->n = v->cap = 0; }
static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}
static void iv_sort(ivec *v) { if (v->n > 1) qsort(v->a, (size_t)v->n, sizeof(int32_t), cmp_i32); }
/* remove every occurrence of x (lists hold each value at most once) */
static void iv_remove(ivec *v, int32_t x) {
    int32_t k = 0;
    for (int32_t t = 0; t < v->n; ++t) if (v->a[t] != x) v->a[k++] = v->a[t];
    v->n = k;
}

/* ------------------------------------------------------------------ */
/* binary min-heap of (degree, index) pairs, lexicographic            */
/* ------------------------------------------------------------------ */
typedef struct { int64_t deg; int32_t idx; } hent;
typedef struct { hent *h; int64_t n, cap; } heap;

static int hless(hent a, hent b) { return a.deg < b.deg || (a.deg == b.deg && a.idx < b.idx); }
static int heap_push(heap *H, int64_t deg, int32_t idx) {
    if (H->n == H->cap) {
        int64_t nc = H->cap ? 2 * H->cap : 64;
        hent *nh = (hent *)realloc(H->h, (size_t)nc * sizeof(hent));
        if (!nh) return -1;
        H->h = nh; H->cap = nc;
    }
    int64_t k = H->n++;
    H->h[k].deg = deg; H->h[k].idx = idx;
    while (k > 0) {
        int64_t par = (k - 1) / 2;
        if (!hless(H->h[k], H->h[par])) break;
        hent t = H->h[k]; H->h[k] = H->h[par]; H->h[par] = t; k = par;
    }
    return 0;
}
static hent heap_pop(heap *H) {
    hent top = H->h[0];
    H->h[0] = H->h[--H->n];
    int64_t k = 0;
    for (;;) {
        int64_t l = 2 * k + 1, r = l + 1, s = k;
        if (l < H->n && hless(H->h[l], H->h[s])) s = l;
        if (r < H->n && hless(H->h[r], H->h[s])) s = r;
        if (s == k) break;
        hent t = H->h[k]; H->h[k] = H->h[s]; H->h[s] = t; k = s;
    }
    return top;
}

/* comparator context for the supervariable test (the oracle is single-threaded) */
static const ivec *g_A, *g_E;
static int cmp_list(const ivec *x, const ivec *y) {
    if (x->n != y->n) return (x->n > y->n) - (x->n < y->n);
    for (int32_t t = 0; t < x->n; ++t)
        if (x->a[t] != y->a[t]) return (x->a[t] > y->a[t]) - (x->a[t] < y->a[t]);
    return 0;
}
static int same_key(int32_t i, int32_t j) {
    return cmp_list(&g_A[i], &g_A[j]) == 0 && cmp_list(&g_E[i], &g_E[j]) == 0;
}
static int cmp_key_then_index(const void *x, const void *y) {
    int32_t i = *(const int32_t *)x, j = *(const int32_t *)y;
    if (g_A[i].n != g_A[j].n) return (g_A[i].n > g_A[j].n) - (g_A[i].n < g_A[j].n);
    if (g_E[i].n != g_E[j].n) return (g_E[i].n > g_E[j].n) - (g_E[i].n < g_E[j].n);
    int c = cmp_list(&g_A[i], &g_A[j]);
    if (c) return c;
    c = cmp_list(&g_E[i], &g_E[j]);
    if (c) return c;
    return (i > j) - (i < j);
}

/* ------------------------------------------------------------------ */
/* Minimum degree on the quotient graph                               */
/* ------------------------------------------------------------------ */
/*
 * The rule (our own specification; the paper leaves the reordering to its
 * sparse solver, Sec. 2.2):
 *
 *   State: principal variables i with weight nv[i], variable list A[i] and
 *   element list E[i]; elements e with variable list L[e].  Initially every
 *   node is a principal variable of weight 1 with A[i] = its graph neighbours,
 *   E[i] empty and d(i) = |A[i]|.  W(S) denotes the sum of nv over a set S.
 *
 *   Repeat until no principal variable is left:
 *    1. pivot p = principal variable of least (d, index);
 *    2. append the members of p (original nodes, increasing) to the order;
 *    3. Lp = (A[p] U union_{e in E[p]} L[e]) \ {p}; the elements of E[p]
 *       are absorbed; p becomes an element with L[p] = Lp;
 *    4. for i in Lp: E[i] <- (E[i] \ E[p]) U {p};  A[i] <- A[i] \ (Lp U {p});
 *    5. among Lp, variables with identical A and identical E are merged
 *       into the one of smallest index (weights add, members concatenate);
 *       the merged ones leave every A and L list;
 *    6. for every principal variable i left in Lp, with rem = total weight
 *       of the principal variables still uneliminated and lp = W(Lp) - nv[i]:
 *         approximate mode (the product rule):
 *           d(i) <- min( rem - nv[i],  d(i) + lp,
 *                        W(A[i]) + lp + sum_{e in E[i], e != p} W(L[e] \ Lp) )
 *         exact mode (test rule):
 *           d(i) <- W((A[i] U union_{e in E[i]} L[e]) \ {i}).
 *
 * The approximate value is the degree bound of Amestoy, Davis and Duff's
 * approximate minimum degree method (without aggressive absorption); it is
 * an upper bound on the exact external degree, which the tests check.
 * With ``merge`` = 0 and exact mode the result is plain minimum degree on the
 * explicit elimination graph, which the tests check against brute force.
 *
 * Input: symmetric graph (both triangles, no self loops) in CSC form.
 * Output: order[k] = node eliminated k-th.  If ``check`` is non-NULL, the
 * exact external degree is also computed in approximate mode and *check
 * counts the updates where the bound fell below it (must stay 0).
 * Returns 0, or a negative value on allocation failure.
 */
int or_min_degree(int32_t N, const int64_t *Gp, const int32_t *Gi, int32_t merge, int32_t exact,
                  int32_t *order, int64_t *check)
{
    int rc = -1;
    ivec *A = (ivec *)calloc((size_t)N, sizeof(ivec));
    ivec *E = (ivec *)calloc((size_t)N, sizeof(ivec));
    ivec *L = (ivec *)calloc((size_t)N, sizeof(ivec));
    ivec *mem = (ivec *)calloc((size_t)N, sizeof(ivec));
    int64_t *nv = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    int64_t *deg = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    int8_t *status = (int8_t *)calloc((size_t)N, 1); /* 0 var, 1 merged, 2 element, 3 absorbed */
    int64_t *mark = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    int64_t *mark2 = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    int32_t *lp = (int32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    heap H = {0};
    int64_t stamp = 0;
    int32_t nord = 0;
    if (!A || !E || !L || !mem || !nv || !deg || !status || !mark || !mark2 || !lp) goto done;
    int64_t rem = N;
    if (check) *check = 0;

    for (int32_t i = 0; i < N; ++i) {
        nv[i] = 1;
        if (iv_push(&mem[i], i)) goto done;
        for (int64_t t = Gp[i]; t < Gp[i + 1]; ++t)
            if (Gi[t] != i && iv_push(&A[i], Gi[t])) goto done;
        iv_sort(&A[i]);
    }
    for (int32_t i = 0; i < N; ++i) {
        int64_t d = 0;
        for (int32_t t = 0; t < A[i].n; ++t) d += nv[A[i].a[t]];
        deg[i] = d;
        if (heap_push(&H, d, i)) goto done;
    }

    while (H.n > 0) {
        hent top = heap_pop(&H);
        int32_t p = top.idx;
        if (status[p] != 0 || deg[p] != top.deg) continue;   /* stale entry */

        /* step 2 */
        int64_t nv_p = nv[p];
        for (int32_t t = 0; t < mem[p].n; ++t) order[nord++] = mem[p].a[t];

        /* step 3: Lp */
        ++stamp;
        int32_t nlp = 0;
        mark[p] = stamp;
        for (int32_t t = 0; t < A[p].n; ++t) {
            int32_t v = A[p].a[t];
            if (status[v] == 0 && mark[v] != stamp) { mark[v] = stamp; lp[nlp++] = v; }
        }
        for (int32_t t = 0; t < E[p].n; ++t) {
            int32_t e = E[p].a[t];
            for (int32_t u = 0; u < L[e].n; ++u) {
                int32_t v = L[e].a[u];
                if (status[v] == 0 && mark[v] != stamp) { mark[v] = stamp; lp[nlp++] = v; }
            }
        }
        qsort(lp, (size_t)nlp, sizeof(int32_t), cmp_i32);
        for (int32_t t = 0; t < E[p].n; ++t) { status[E[p].a[t]] = 3; iv_free(&L[E[p].a[t]]); }
        status[p] = 2;
        iv_free(&A[p]); iv_free(&E[p]);
        for (int32_t t = 0; t < nlp; ++t) if (iv_push(&L[p], lp[t])) goto done;

        /* step 4 (mark[v]==stamp identifies Lp members and p itself) */
        for (int32_t t = 0; t < nlp; ++t) {
            int32_t i = lp[t];
            int32_t k = 0;
            for (int32_t u = 0; u < E[i].n; ++u)
                if (status[E[i].a[u]] == 2) E[i].a[k++] = E[i].a[u];
            E[i].n = k;
            if (iv_push(&E[i], p)) goto done;
            iv_sort(&E[i]);
            k = 0;
            for (int32_t u = 0; u < A[i].n; ++u)
                if (mark[A[i].a[u]] != stamp) A[i].a[k++] = A[i].a[u];
            A[i].n = k;
        }

        /* step 5: merge indistinguishable variables of Lp.  Sort Lp by
         * (|A|, |E|, A, E, index); every run of equal keys merges into its
         * first member, the one of smallest index. */
        if (merge && nlp > 1) {
            g_A = A; g_E = E;
            qsort(lp, (size_t)nlp, sizeof(int32_t), cmp_key_then_index);
            int32_t t = 0;
            while (t < nlp) {
                int32_t r = lp[t], u = t + 1;
                while (u < nlp && same_key(r, lp[u])) ++u;
                for (int32_t w = t + 1; w < u; ++w) {
                    int32_t j = lp[w];
                    nv[r] += nv[j];
                    for (int32_t x = 0; x < mem[j].n; ++x) if (iv_push(&mem[r], mem[j].a[x])) goto done;
                    iv_free(&mem[j]);
                    for (int32_t x = 0; x < A[j].n; ++x) iv_remove(&A[A[j].a[x]], j);
                    for (int32_t x = 0; x < E[j].n; ++x) iv_remove(&L[E[j].a[x]], j);
                    iv_free(&A[j]); iv_free(&E[j]);
                    status[j] = 1; nv[j] = 0;
                }
                if (u - t > 1) iv_sort(&mem[r]);
                t = u;
            }
            qsort(lp, (size_t)nlp, sizeof(int32_t), cmp_i32);
        }

        /* step 6: degree update */
        rem -= nv_p;
        {
            int64_t wlp = 0;
            for (int32_t t = 0; t < nlp; ++t) if (status[lp[t]] == 0) wlp += nv[lp[t]];
            /* mark the surviving members of Lp */
            ++stamp;
            int64_t lpstamp = stamp;
            for (int32_t t = 0; t < nlp; ++t) if (status[lp[t]] == 0) mark[lp[t]] = lpstamp;
            for (int32_t t = 0; t < nlp; ++t) {
                int32_t i = lp[t];
                if (status[i] != 0) continue;
                int64_t lpi = wlp - nv[i];
                int64_t dex = -1;
                if (exact || check) {
                    ++stamp;
                    mark2[i] = stamp;
                    dex = 0;
                    for (int32_t u = 0; u < A[i].n; ++u) {
                        int32_t v = A[i].a[u];
                        if (mark2[v] != stamp) { mark2[v] = stamp; dex += nv[v]; }
                    }
                    for (int32_t u = 0; u < E[i].n; ++u) {
                        int32_t e = E[i].a[u];
                        for (int32_t w = 0; w < L[e].n; ++w) {
                            int32_t v = L[e].a[w];
                            if (mark2[v] != stamp) { mark2[v] = stamp; dex += nv[v]; }
                        }
                    }
                }
                int64_t d;
                if (exact) {
                    d = dex;
                } else {
                    int64_t wa = 0, we = 0;
                    for (int32_t u = 0; u < A[i].n; ++u) wa += nv[A[i].a[u]];
                    for (int32_t u = 0; u < E[i].n; ++u) {
                        int32_t e = E[i].a[u];
                        if (e == p) continue;
                        for (int32_t w = 0; w < L[e].n; ++w) {
                            int32_t v = L[e].a[w];
                            if (mark[v] != lpstamp) we += nv[v];
                        }
                    }
                    int64_t b1 = rem - nv[i], b2 = deg[i] + lpi, b3 = wa + lpi + we;
                    d = b1 < b2 ? b1 : b2;
                    if (b3 < d) d = b3;
                    if (check && d < dex) *check += 1;
                }
                deg[i] = d;
                if (heap_push(&H, d, i)) goto done;
            }
        }
    }
    rc = (nord == N) ? 0 : -2;
done:
    if (A) for (int32_t i = 0; i < N; ++i) iv_free(&A[i]);
    if (E) for (int32_t i = 0; i < N; ++i) iv_free(&E[i]);
    if (L) for (int32_t i = 0; i < N; ++i) iv_free(&L[i]);
    if (mem) for (int32_t i = 0; i < N; ++i) iv_free(&mem[i]);
    free(A); free(E); free(L); free(mem); free(nv); free(deg); free(status); free(mark); free(mark2); free(lp);
    free(H.h);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Elimination tree of a symmetric matrix given by its upper triangle  */
/* ------------------------------------------------------------------ */
/*
 * parent[j] = min { i > j : L_ij != 0 }, or -1.  Textbook algorithm with
 * path compression over the upper-triangular columns (Liu's algorithm).
 */
int or_etree(int32_t N, const int64_t *Up, const int32_t *Ui, int32_t *parent)
{
    int32_t *anc = (int32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    if (!anc) return -1;
    for (int32_t k = 0; k < N; ++k) {
        parent[k] = -1; anc[k] = -1;
        for (int64_t t = Up[k]; t < Up[k + 1]; ++t) {
            int32_t i = Ui[t];
            while (i != -1 && i < k) {
                int32_t next = anc[i];
                anc[i] = k;
                if (next == -1) { parent[i] = k; break; }
                i = next;
            }
        }
    }
    free(anc);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Pattern of L (strictly lower part, CSC) via row subtrees            */
/* ------------------------------------------------------------------ */
/*
 * Row k of L has a nonzero in column j < k exactly when j lies on an etree
 * path from some i with A_ik != 0 (i < k) up to (but excluding) k.
 * Pass 1 (Li == NULL): counts per column into cnt[N] (strictly lower).
 * Pass 2: writes the row indices; rows come out sorted because k increases.
 */
int or_lpattern(int32_t N, const int64_t *Up, const int32_t *Ui, const int32_t *parent,
                const int64_t *Lp, int64_t *cnt, int32_t *Li)
{
    int32_t *flag = (int32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    int64_t *pos = (int64_t *)calloc((size_t)(N > 0 ? N : 1), sizeof(int64_t));
    if (!flag || !pos) { free(flag); free(pos); return -1; }
    for (int32_t j = 0; j < N; ++j) { flag[j] = -1; cnt[j] = 0; }
    for (int32_t k = 0; k < N; ++k) {
        flag[k] = k;
        for (int64_t t = Up[k]; t < Up[k + 1]; ++t) {
            int32_t i = Ui[t];
            if (i >= k) continue;
            while (flag[i] != k) {
                flag[i] = k;
                cnt[i] += 1;
                if (Li) { Li[Lp[i] + pos[i]] = k; pos[i] += 1; }
                i = parent[i];
            }
        }
    }
    free(flag); free(pos);
    return 0;
}

/*
 * Work of each row of the up-looking factorization below, from the same row
 * subtrees: row k has an entry in column i for each i on those paths, and
 * that entry is the t-th of column i (t = entries of column i in rows < k),
 * whose update costs t multiply-adds; with one division per entry and one
 * for the pivot, rowops[k] = 1 + sum over the row's entries of (t + 1).
 * rowcnt[k] = entries of row k.  Used to time a bounded prefix of a large
 * factorization and scale it to the whole.
 */
int or_row_work(int32_t N, const int64_t *Up, const int32_t *Ui, const int32_t *parent,
                int64_t *rowcnt, double *rowops)
{
    int32_t *flag = (int32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    int64_t *cnt = (int64_t *)calloc((size_t)(N > 0 ? N : 1), sizeof(int64_t));
    if (!flag || !cnt) { free(flag); free(cnt); return -1; }
    for (int32_t j = 0; j < N; ++j) flag[j] = -1;
    for (int32_t k = 0; k < N; ++k) {
        double ops = 1.0;
        int64_t nk = 0;
        flag[k] = k;
        for (int64_t t = Up[k]; t < Up[k + 1]; ++t) {
            int32_t i = Ui[t];
            if (i >= k) continue;
            while (flag[i] != k) {
                flag[i] = k;
                ops += (double)cnt[i] + 1.0;
                cnt[i] += 1;
                nk += 1;
                i = parent[i];
            }
        }
        rowcnt[k] = nk;
        rowops[k] = ops;
    }
    free(flag); free(cnt);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Up-looking numeric LDL' on a known pattern                          */
/* ------------------------------------------------------------------ */
/*
 * Factors the symmetric matrix whose upper triangle is (Up, Ui, Ux) (columns
 * with sorted rows, diagonal present) as L D L' with unit lower L, no
 * pivoting.  Row k of L is obtained by a sparse triangular solve over the
 * row-k pattern (processed in increasing column order, which respects the
 * etree), then d_k = a_kk - sum_j L_kj^2 d_j.
 *
 * Dynamic regularization: if sign[k] * d_k <= eps then d_k = sign[k] * delta
 * (sign[k] = +1 for primal rows, -1 for dual rows).  The number of such
 * events is returned in *nreg.
 *
 * Lp/Li: the strictly-lower pattern from or_lpattern.  Lx receives values in
 * that pattern's positions, D the diagonal.  Returns 0, -1 on allocation
 * failure, -3 on a non-finite pivot.
 */
int or_ldl_numeric_rows(int32_t N, int32_t k_end, const int64_t *Up, const int32_t *Ui,
                        const double *Ux, const int32_t *parent, const int64_t *Lp,
                        const int32_t *Li, const int8_t *sign, double eps, double delta,
                        double *Lx, double *D, int64_t *nreg);

int or_ldl_numeric(int32_t N, const int64_t *Up, const int32_t *Ui, const double *Ux,
                   const int32_t *parent, const int64_t *Lp, const int32_t *Li,
                   const int8_t *sign, double eps, double delta,
                   double *Lx, double *D, int64_t *nreg)
{
    return or_ldl_numeric_rows(N, N, Up, Ui, Ux, parent, Lp, Li, sign, eps, delta, Lx, D, nreg);
}

int or_ldl_numeric_rows_marked(int32_t N, int32_t k_end, int32_t k_mark, const int64_t *Up,
                               const int32_t *Ui, const double *Ux, const int32_t *parent,
                               const int64_t *Lp, const int32_t *Li, const int8_t *sign, double eps,
                               double delta, double *Lx, double *D, int64_t *nreg, double *t_mark);

/* The same factorization stopped after rows 0..k_end-1 (used to time a
 * bounded sample of a large factorization). */
int or_ldl_numeric_rows(int32_t N, int32_t k_end, const int64_t *Up, const int32_t *Ui,
                        const double *Ux, const int32_t *parent, const int64_t *Lp,
                        const int32_t *Li, const int8_t *sign, double eps, double delta,
                        double *Lx, double *D, int64_t *nreg)
{
    return or_ldl_numeric_rows_marked(N, k_end, -1, Up, Ui, Ux, parent, Lp, Li, sign, eps, delta, Lx, D,
                                      nreg, NULL);
}

/* Seconds of a monotonic clock. */
static double or_now(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* The same, with the clock read when row k_mark starts (*t_mark, seconds
 * since the call started; untouched when k_mark is outside 0..k_end-1): the
 * work of a stretch of rows can then be timed inside one run. */
int or_ldl_numeric_rows_marked(int32_t N, int32_t k_end, int32_t k_mark, const int64_t *Up,
                               const int32_t *Ui, const double *Ux, const int32_t *parent,
                               const int64_t *Lp, const int32_t *Li, const int8_t *sign, double eps,
                               double delta, double *Lx, double *D, int64_t *nreg, double *t_mark)
{
    const double t0 = or_now();
    double *y = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    int32_t *flag = (int32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    int32_t *patt = (int32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)calloc((size_t)(N > 0 ? N : 1), sizeof(int64_t));
    int rc = 0;
    if (!y || !flag || !patt || !fill) { rc = -1; goto done; }
    *nreg = 0;
    for (int32_t j = 0; j < N; ++j) flag[j] = -1;
    for (int32_t k = 0; k < k_end; ++k) {
        if (k == k_mark && t_mark) *t_mark = or_now() - t0;
        /* scatter column k of the upper triangle; collect the row-k pattern */
        int32_t np = 0;
        double akk = 0.0;
        flag[k] = k;
        for (int64_t t = Up[k]; t < Up[k + 1]; ++t) {
            int32_t i = Ui[t];
            if (i == k) { akk += Ux[t]; continue; }
            y[i] += Ux[t];
            while (flag[i] != k) { flag[i] = k; patt[np++] = i; i = parent[i]; }
        }
        qsort(patt, (size_t)np, sizeof(int32_t), cmp_i32);
        /* sparse solve L(0:k,0:k) D w = a(0:k,k), column by column */
        double dk = akk;
        for (int32_t t = 0; t < np; ++t) {
            int32_t j = patt[t];
            double yj = y[j];
            y[j] = 0.0;
            /* entries of column j computed so far are rows < k */
            for (int64_t u = Lp[j]; u < Lp[j] + fill[j]; ++u) y[Li[u]] -= Lx[u] * yj;
            double lkj = yj / D[j];
            dk -= lkj * yj;
            Lx[Lp[j] + fill[j]] = lkj;      /* row k is the next row of column j */
            fill[j] += 1;
        }
        if (!isfinite(dk)) { rc = -3; goto done; }
        if ((double)sign[k] * dk <= eps) { dk = (double)sign[k] * delta; *nreg += 1; }
        D[k] = dk;
    }
done:
    free(y); free(flag); free(patt); free(fill);
    return rc;
}

/* Solve L D L' x = b in place (all in the permuted ordering). */
int or_ldl_solve(int32_t N, const int64_t *Lp, const int32_t *Li, const double *Lx,
                 const double *D, double *x)
{
    for (int32_t j = 0; j < N; ++j)
        for (int64_t u = Lp[j]; u < Lp[j + 1]; ++u) x[Li[u]] -= Lx[u] * x[j];
    for (int32_t j = 0; j < N; ++j) x[j] /= D[j];
    for (int32_t j = N - 1; j >= 0; --j)
        for (int64_t u = Lp[j]; u < Lp[j + 1]; ++u) x[j] -= Lx[u] * x[Li[u]];
    return 0;
}
