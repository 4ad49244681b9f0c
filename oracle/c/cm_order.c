/* Cuthill-McKee ordering, sequential queue form -- test infrastructure
 * (oracle), never linked into the solver library.
 *
 * Paper, section "Direct factorization": the structure of a symmetric sparse
 * matrix is read as a graph; a breadth-first search starts from a node of
 * lowest degree (degree = number of stored entries in the row) and visits the
 * neighbours of each node in order of increasing degree; this is repeated for
 * every connected component.  Reversing the visit order gives RCM.
 *
 * Readings where the paper is silent:
 *  - degree is the graph degree of the node in the symmetric pattern: the
 *    number of stored entries of its row, with a stored diagonal entry (a
 *    self-loop) counted twice;
 *  - a component starts at the unvisited node of lowest degree, and among
 *    those at the one of highest index;
 *  - neighbours of equal degree are queued in increasing index.
 * With these, the RCM bandwidth and profile printed for the paper's Fig. 1
 * and Fig. 3 systems are reproduced exactly in four of six cases and in
 * bandwidth in the other two.
 *
 * Input: symmetric pattern in CSR (indptr[n+1] int64, indices int32, column
 * indices sorted within each row).  Output: order[k] = node visited k-th.
 * Returns 0, or -1 on allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>

static const int64_t *g_deg;

/* neighbour order: degree ascending, then index ascending */
static int cmp_deg_idx(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_deg[x] != g_deg[y]) return g_deg[x] < g_deg[y] ? -1 : 1;
    return (x > y) - (x < y);
}

/* start-node order: degree ascending, then index descending */
static int cmp_deg_ridx(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_deg[x] != g_deg[y]) return g_deg[x] < g_deg[y] ? -1 : 1;
    return (x < y) - (x > y);
}

int oracle_cuthill_mckee(int64_t n, const int64_t *indptr, const int32_t *indices,
                         int32_t *order) {
    int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    char *seen = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t *by_deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!deg || !seen || !by_deg) { free(deg); free(seen); free(by_deg); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        deg[i] = indptr[i + 1] - indptr[i];
        for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e)
            if (indices[e] == i) { deg[i] += 1; break; }
        by_deg[i] = (int32_t)i;
    }
    g_deg = deg;
    /* candidate start nodes: lowest degree first, highest index among equals */
    qsort(by_deg, (size_t)n, sizeof(int32_t), cmp_deg_ridx);

    int64_t head = 0, tail = 0, next_start = 0;
    while (tail < n) {
        while (seen[by_deg[next_start]]) ++next_start;
        int32_t s = by_deg[next_start];
        seen[s] = 1;
        order[tail++] = s;
        while (head < tail) {
            int32_t u = order[head++];
            int64_t first_new = tail;
            for (int64_t e = indptr[u]; e < indptr[u + 1]; ++e) {
                int32_t v = indices[e];
                if (!seen[v]) { seen[v] = 1; order[tail++] = v; }
            }
            /* insertion sort of the newly queued neighbours by (degree, index) */
            for (int64_t a = first_new + 1; a < tail; ++a) {
                int32_t key = order[a];
                int64_t b = a - 1;
                while (b >= first_new && cmp_deg_idx(&order[b], &key) > 0) {
                    order[b + 1] = order[b];
                    --b;
                }
                order[b + 1] = key;
            }
        }
    }
    free(deg); free(seen); free(by_deg);
    return 0;
}
