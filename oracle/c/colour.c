/* Greedy vertex colouring in a given visit order -- test infrastructure
 * (oracle), never linked into the solver library.
 *
 * Not a step of the paper.  The ILU preconditioner of section "Iterative
 * Solvers" is applied by forward and backward substitution, and in RCM order
 * (section "Direct factorization") those substitutions form long chains of
 * dependent rows.  Numbering the unknowns colour class by colour class, for
 * a proper colouring of the structure of A + A^T, puts every off-diagonal
 * entry of A between two different classes, so a zero-fill factor has at
 * most as many dependent steps per substitution as there are colours.
 *
 * Definition (the textbook sequential greedy colouring): visit the vertices
 * in the given order and give each the smallest non-negative colour that no
 * already visited neighbour carries.  A stored diagonal entry (self-loop) is
 * not an edge.
 *
 * Input: symmetric pattern in CSR (indptr[n+1] int64, indices int32) and the
 * visit order order[k] = vertex visited k-th (a permutation of 0..n-1).
 * Output: colour[v].  Returns the number of colours used, or -1 on
 * allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>

int oracle_greedy_colour(int64_t n, const int64_t *indptr, const int32_t *indices, const int32_t *order,
                         int32_t *colour) {
    /* taken[c] == k: colour c is carried by a visited neighbour of the k-th
     * vertex (a vertex has at most n - 1 neighbours, so colours stay < n) */
    int64_t *taken = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!taken) return -1;
    for (int64_t i = 0; i < n; ++i) colour[i] = -1;
    for (int64_t c = 0; c <= n; ++c) taken[c] = -1;
    int32_t used = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int32_t v = order[k];
        for (int64_t e = indptr[v]; e < indptr[v + 1]; ++e) {
            const int32_t u = indices[e];
            if (u != v && colour[u] >= 0) taken[colour[u]] = k;
        }
        int32_t c = 0;
        while (taken[c] == k) ++c;
        colour[v] = c;
        if (c + 1 > used) used = c + 1;
    }
    free(taken);
    return used;
}
