/*
 * CPU oracle for betweenness centrality -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path (libmfbc) never calls it and the
 * two share no code.
 *
 * What it computes (Section 2.4, Table 1 of Solomonik, Besta, Vella,
 * Hoefler, "Scaling Betweenness Centrality using Communication-Efficient
 * Sparse Matrix Multiplication", SC17):
 *   tau(s,v)    shortest-path distance from s to v (weights >= 1, integers);
 *   sigma(s,v)  number of shortest s->v paths, sigma(s,s) = 1;
 *   delta(s,v)  = sum_t sigma(s,t,v) / sigma(s,t), with sigma(s,t,s) =
 *               sigma(s,t,t) = 0, so delta(s,s) = 0;
 *   lambda(v)   = sum over the listed sources s of delta(s,v)
 *               (ordered pairs, no halving, no normalisation).
 * It follows Brandes' two-phase scheme described in Section 2.4: a
 * single-source search (breadth-first for unweighted graphs, Dijkstra with a
 * binary heap for weighted ones) that records distances, path counts and the
 * order in which vertices are settled, then a sweep in reverse settling order
 * that accumulates the dependency recurrence over the successors w of v on
 * shortest paths (w is a successor of v when tau(s,v) + A(v,w) = tau(s,w)):
 *     delta(s,v) = sum_w sigma(s,v)/sigma(s,w) * (1 + delta(s,w)).
 * Arithmetic is IEEE binary64; distances are int64.  Arcs are read as
 * out-arcs (row u of the CSR lists the heads of u's arcs), so directed graphs
 * work unchanged; for an undirected graph the CSR is symmetric.
 *
 * It also reports, for the frontier checks, the height of each reachable
 * vertex in the shortest-path DAG of s: 0 for a vertex with no successor,
 * else 1 + the largest height among its successors.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORACLE_INF INT64_MAX

typedef struct {
    int64_t d;
    int32_t v;
} hitem;

typedef struct {
    hitem *a;
    int64_t size, cap;
} heap_t;

static int heap_push(heap_t *h, int64_t d, int32_t v) {
    if (h->size == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        hitem *na = (hitem *)realloc(h->a, (size_t)nc * sizeof(hitem));
        if (!na) return -1;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->size++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p].d <= d) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].d = d;
    h->a[i].v = v;
    return 0;
}

static hitem heap_pop(heap_t *h) {
    hitem top = h->a[0];
    hitem last = h->a[--h->size];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= h->size) break;
        if (c + 1 < h->size && h->a[c + 1].d < h->a[c].d) c++;
        if (h->a[c].d >= last.d) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->size > 0) h->a[i] = last;
    return top;
}

/* Per-thread work arrays. */
typedef struct {
    int64_t *dist;
    double *sigma, *delta;
    int32_t *order, *height;
    char *done;
    heap_t heap;
} work_t;

/* Single-source search; returns the number of settled vertices (in order[]). */
static int64_t search(int32_t n, const int64_t *rp, const int32_t *col, const int32_t *w,
                      int32_t s, work_t *k) {
    for (int32_t v = 0; v < n; v++) {
        k->dist[v] = ORACLE_INF;
        k->sigma[v] = 0.0;
        k->done[v] = 0;
    }
    k->dist[s] = 0;
    k->sigma[s] = 1.0;
    int64_t cnt = 0;
    if (w == NULL) {
        /* breadth-first search: order[] doubles as the FIFO queue */
        int64_t head = 0;
        k->order[cnt++] = s;
        while (head < cnt) {
            int32_t v = k->order[head++];
            int64_t dn = k->dist[v] + 1;
            for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
                int32_t x = col[e];
                if (k->dist[x] == ORACLE_INF) {
                    k->dist[x] = dn;
                    k->order[cnt++] = x;
                }
                if (k->dist[x] == dn) k->sigma[x] += k->sigma[v];
            }
        }
    } else {
        /* Dijkstra with a binary heap and lazy deletion */
        k->heap.size = 0;
        heap_push(&k->heap, 0, s);
        while (k->heap.size > 0) {
            hitem it = heap_pop(&k->heap);
            int32_t v = it.v;
            if (k->done[v] || it.d != k->dist[v]) continue;
            k->done[v] = 1;
            k->order[cnt++] = v;
            for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
                int32_t x = col[e];
                int64_t nd = k->dist[v] + (int64_t)w[e];
                if (nd < k->dist[x]) {
                    k->dist[x] = nd;
                    k->sigma[x] = k->sigma[v];
                    heap_push(&k->heap, nd, x);
                } else if (nd == k->dist[x]) {
                    k->sigma[x] += k->sigma[v];
                }
            }
        }
    }
    return cnt;
}

/* Reverse sweep: delta and heights from the successors of each vertex. */
static void dependencies(const int64_t *rp, const int32_t *col, const int32_t *w,
                         int64_t cnt, work_t *k) {
    for (int64_t i = cnt - 1; i >= 0; i--) {
        int32_t v = k->order[i];
        double acc = 0.0;
        int32_t h = 0;
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            int32_t x = col[e];
            int64_t wt = w ? (int64_t)w[e] : 1;
            if (k->dist[x] != ORACLE_INF && k->dist[v] + wt == k->dist[x]) {
                acc += k->sigma[v] / k->sigma[x] * (1.0 + k->delta[x]);
                if (k->height[x] + 1 > h) h = k->height[x] + 1;
            }
        }
        k->delta[v] = acc;
        k->height[v] = h;
    }
}

/*
 * oracle_bc: lambda over the listed sources, plus optional per-source outputs.
 *   n, rp[n+1], col[arcs], w[arcs] or NULL (all weights 1): out-arc CSR.
 *   sources[n_src]: each in [0,n); repeats are counted per occurrence.
 *   lambda_out[n]: overwritten with sum_s delta(s,.) (delta(s,s) excluded).
 *   dist_out / sigma_out / delta_out / height_out: NULL or [n_src][n]
 *     (dist -1 and height -1 for unreachable; delta(s,s) reported as 0).
 *   nthreads <= 0 uses OpenMP's default.
 * Returns 0, or -1 on allocation failure or a bad source.
 */
int oracle_bc(int32_t n, const int64_t *rp, const int32_t *col, const int32_t *w,
              const int32_t *sources, int64_t n_src, double *lambda_out,
              int64_t *dist_out, double *sigma_out, double *delta_out,
              int32_t *height_out, int32_t nthreads) {
    for (int64_t i = 0; i < n_src; i++)
        if (sources[i] < 0 || sources[i] >= n) return -1;
    int T = nthreads > 0 ? nthreads : omp_get_max_threads();
    double *lam = (double *)calloc((size_t)T * (size_t)n, sizeof(double));
    if (!lam) return -1;
    int failed = 0;
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        work_t k;
        memset(&k, 0, sizeof(k));
        k.dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        k.sigma = (double *)malloc((size_t)n * sizeof(double));
        k.delta = (double *)malloc((size_t)n * sizeof(double));
        k.order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        k.height = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        k.done = (char *)malloc((size_t)n);
        if (!k.dist || !k.sigma || !k.delta || !k.order || !k.height || !k.done) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp barrier
        int any_failed;
#pragma omp atomic read
        any_failed = failed;
        if (!any_failed) {
            /* every thread takes this branch or none does: the loop's
               implicit barrier is reached by the whole team */
            double *my = lam + (size_t)t * (size_t)n;
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n_src; i++) {
                int32_t s = sources[i];
                int64_t cnt = search(n, rp, col, w, s, &k);
                dependencies(rp, col, w, cnt, &k);
                for (int64_t j = 0; j < cnt; j++) {
                    int32_t v = k.order[j];
                    if (v != s) my[v] += k.delta[v];
                }
                if (dist_out || sigma_out || delta_out || height_out) {
                    size_t off = (size_t)i * (size_t)n;
                    for (int32_t v = 0; v < n; v++) {
                        int reach = k.dist[v] != ORACLE_INF;
                        if (dist_out) dist_out[off + v] = reach ? k.dist[v] : -1;
                        if (sigma_out) sigma_out[off + v] = k.sigma[v];
                        if (delta_out) delta_out[off + v] = (reach && v != s) ? k.delta[v] : 0.0;
                        if (height_out) height_out[off + v] = reach ? k.height[v] : -1;
                    }
                }
            }
        }
        free(k.dist);
        free(k.sigma);
        free(k.delta);
        free(k.order);
        free(k.height);
        free(k.done);
        free(k.heap.a);
    }
    if (failed) {
        free(lam);
        return -1;
    }
    /* fixed summation order over threads */
    for (int32_t v = 0; v < n; v++) {
        double acc = 0.0;
        for (int t = 0; t < T; t++) acc += lam[(size_t)t * (size_t)n + v];
        lambda_out[v] = acc;
    }
    free(lam);
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
