/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of the real-scheme
 * extraction for T-curves ("Fast Isotopy Computation for T-Curves",
 * Sec. 2, Algorithm 1).  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; the product path
 * (the HIP library) never links, calls or includes it, and shares no code
 * with it.
 *
 * Every step follows the paper in its own order and notation:
 *   O0  validate the triangulation (Sec. 2: unimodular = every triangle has
 *       area 1/2, represented by its edge list)
 *   O1  build the diamond A<> and E(T<>) by reflecting into four quadrants
 *       (Alg. 1, first step)
 *   O2  extend sigma to A<> by eq. (signs) (Alg. 1, second step)
 *   O3  crossed edges: endpoints of distinct signs (Sec. 2)
 *   O4  components: connected components of the non-crossed subgraph
 *       (Alg. 1, "components and regions")
 *   O5  regions: components merged along antipodal boundary pairs
 *       (i,d-i)~-(i,d-i), (i,i-d)~-(i,i-d) (Sec. 2)
 *   O6  region adjacency graph from crossed edges (Alg. 1, "root and real
 *       scheme"; Sec. 2 definition: one edge per curve component, a
 *       self-loop when both sides coincide)
 *   O7  root: odd d -> the unique region holding two crossed-edge-adjacent
 *       components; even d -> the unique region whose components form an
 *       odd cycle under antipodal adjacency (Alg. 1; proof of Thm. 2)
 *   O8  the adjacency graph is a tree (proof of Thm. 2)
 *   O9  canonical form of the rooted tree (Alg. 1, last step; AHU encoding,
 *       proof of Thm. 2).  The paper fixes no encoding; this project's
 *       encoding is:  c(v) = '1' . concat(c(children) sorted descending,
 *       '1' > '0') . '0';  W = concat of the sorted codes of the root's
 *       children;  code = 2^|W| + int(W) (first character of W is the most
 *       significant bit), bit 127 set iff d is odd (the pseudo-line J).
 *
 * Conventions (not fixed by the paper):
 *   lattice point order k(i,j) = j(d+1) - j(j-1)/2 + i  (row-major by j);
 *   mask bit k = sigma(p_k) in GF(2), 0 = '+' (coefficient sign (-1)^sigma,
 *   Thm. 1); masks are two little-endian 64-bit words (lo, hi).
 *
 * Nothing here is optimised: adjacency is rebuilt per evaluation, components
 * are found by breadth-first search, codes are built as character strings.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OR_OK 0
#define OR_ERR_ARG -1
#define OR_ERR_TRI -2
#define OR_ERR_ASSERT -3

#define DMAX 12

static __thread char g_err[256];

const char *oracle_last_error(void) { return g_err; }

static int fail(int code, const char *msg, int a, int b) {
    snprintf(g_err, sizeof g_err, msg, a, b);
    return code;
}

/* ---- lattice A = d*Delta_2 cap Z^2 (eq. lattice) ---- */

int oracle_n_points(int d) { return (d + 1) * (d + 2) / 2; }

int oracle_point_index(int d, int i, int j) {
    if (i < 0 || j < 0 || i + j > d) return -1;
    return j * (d + 1) - j * (j - 1) / 2 + i;
}

static int in_A(int d, int i, int j) { return i >= 0 && j >= 0 && i + j <= d; }

static int iabs(int x) { return x < 0 ? -x : x; }

static int gcd(int a, int b) {
    a = iabs(a); b = iabs(b);
    while (b) { int t = a % b; a = b; b = t; }
    return a;
}

/* ---- the triangulation T, validated (O0) ---- */

typedef struct {
    int d;
    int n_edges;
    int (*e)[4];          /* i0,j0,i1,j1 */
    int n_tri;
    int (*tri)[3];        /* point indices */
} tri_t;

static void tri_free(tri_t *t) {
    free(t->e); free(t->tri);
    t->e = NULL; t->tri = NULL;
}

/* twice the signed area of (a,b,c) */
static int det3(int ax, int ay, int bx, int by, int cx, int cy) {
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

/* An edge lies on the boundary of d*Delta_2 iff both ends lie on one side. */
static int boundary_edge(int d, int i0, int j0, int i1, int j1) {
    if (j0 == 0 && j1 == 0) return 1;
    if (i0 == 0 && i1 == 0) return 1;
    if (i0 + j0 == d && i1 + j1 == d) return 1;
    return 0;
}

static int tri_build(int d, const int32_t *edges, int n_edges, tri_t *out) {
    memset(out, 0, sizeof *out);
    if (d < 1 || d > DMAX) return fail(OR_ERR_ARG, "degree %d outside [1,12]", d, 0);
    int nA = oracle_n_points(d);
    if (n_edges != nA + d * d - 1)
        return fail(OR_ERR_TRI, "edge count %d, a unimodular triangulation has %d", n_edges, nA + d * d - 1);
    /* adjacency matrix over A, plain */
    unsigned char *adj = calloc((size_t)nA * nA, 1);
    out->d = d;
    out->n_edges = n_edges;
    out->e = malloc(sizeof(int[4]) * n_edges);
    for (int k = 0; k < n_edges; k++) {
        int i0 = edges[4 * k], j0 = edges[4 * k + 1], i1 = edges[4 * k + 2], j1 = edges[4 * k + 3];
        if (!in_A(d, i0, j0) || !in_A(d, i1, j1)) { free(adj); tri_free(out); return fail(OR_ERR_TRI, "edge %d has an endpoint outside A (%d)", k, 0); }
        if (gcd(i1 - i0, j1 - j0) != 1) { free(adj); tri_free(out); return fail(OR_ERR_TRI, "edge %d is not primitive (%d)", k, 0); }
        int a = oracle_point_index(d, i0, j0), b = oracle_point_index(d, i1, j1);
        if (adj[a * nA + b]) { free(adj); tri_free(out); return fail(OR_ERR_TRI, "edge %d is repeated (%d)", k, 0); }
        adj[a * nA + b] = adj[b * nA + a] = 1;
        out->e[k][0] = i0; out->e[k][1] = j0; out->e[k][2] = i1; out->e[k][3] = j1;
    }
    /* coordinates of point k */
    int *pi = malloc(sizeof(int) * nA), *pj = malloc(sizeof(int) * nA);
    for (int j = 0; j <= d; j++)
        for (int i = 0; i + j <= d; i++) { int k = oracle_point_index(d, i, j); pi[k] = i; pj[k] = j; }
    /* triangles: 3-cliques of area 1/2 */
    out->tri = malloc(sizeof(int[3]) * (size_t)(2 * d * d + 8));
    int nt = 0, bad = 0;
    for (int a = 0; a < nA && !bad; a++)
        for (int b = a + 1; b < nA && !bad; b++) {
            if (!adj[a * nA + b]) continue;
            for (int c = b + 1; c < nA; c++) {
                if (!adj[a * nA + c] || !adj[b * nA + c]) continue;
                int D = det3(pi[a], pj[a], pi[b], pj[b], pi[c], pj[c]);
                if (iabs(D) != 1) continue;
                if (nt >= 2 * d * d + 8) { bad = 1; break; }
                out->tri[nt][0] = a; out->tri[nt][1] = b; out->tri[nt][2] = c; nt++;
            }
        }
    out->n_tri = nt;
    if (bad || nt != d * d) {
        free(adj); free(pi); free(pj); tri_free(out);
        return fail(OR_ERR_TRI, "found %d unimodular triangles, need %d", nt, d * d);
    }
    /* every interior edge in exactly two triangles on opposite sides, every
     * boundary edge in exactly one */
    for (int k = 0; k < n_edges; k++) {
        int a = oracle_point_index(d, out->e[k][0], out->e[k][1]);
        int b = oracle_point_index(d, out->e[k][2], out->e[k][3]);
        int cnt = 0, side_sum = 0;
        for (int t = 0; t < nt; t++) {
            int *T = out->tri[t];
            int has_a = (T[0] == a || T[1] == a || T[2] == a);
            int has_b = (T[0] == b || T[1] == b || T[2] == b);
            if (!(has_a && has_b)) continue;
            int c = T[0] + T[1] + T[2] - a - b;
            int D = det3(pi[a], pj[a], pi[b], pj[b], pi[c], pj[c]);
            cnt++;
            side_sum += D;
        }
        int bd = boundary_edge(d, out->e[k][0], out->e[k][1], out->e[k][2], out->e[k][3]);
        if ((bd && cnt != 1) || (!bd && (cnt != 2 || side_sum != 0))) {
            free(adj); free(pi); free(pj); tri_free(out);
            return fail(OR_ERR_TRI, "edge %d lies in %d triangles (not a triangulation)", k, cnt);
        }
    }
    free(adj); free(pi); free(pj);
    return OR_OK;
}

/* ---- the diamond A<> and E(T<>) (O1) ---- */

typedef struct {
    int d, nA;
    int nV;                  /* |A<>| = 2d^2+2d+1 */
    int *vx, *vy;            /* coordinates of diamond vertex v */
    int *vid;                /* (x+d)*(2d+1)+(y+d) -> v, or -1 */
    int nE;                  /* |E(T<>)| = 6d^2+2d (Table 1) */
    int (*E)[2];
    int nP;                  /* antipodal boundary pairs, 2d */
    int (*P)[2];
} diamond_t;

static int dkey(int d, int x, int y) { return (x + d) * (2 * d + 1) + (y + d); }

static void diamond_free(diamond_t *D) {
    free(D->vx); free(D->vy); free(D->vid); free(D->E); free(D->P);
    memset(D, 0, sizeof *D);
}

static int diamond_build(const tri_t *T, diamond_t *D) {
    int d = T->d;
    memset(D, 0, sizeof *D);
    D->d = d;
    D->nA = oracle_n_points(d);
    int side = 2 * d + 1;
    D->vid = malloc(sizeof(int) * side * side);
    for (int k = 0; k < side * side; k++) D->vid[k] = -1;
    D->vx = malloc(sizeof(int) * side * side);
    D->vy = malloc(sizeof(int) * side * side);
    int nV = 0;
    for (int y = -d; y <= d; y++)
        for (int x = -d; x <= d; x++)
            if (iabs(x) + iabs(y) <= d) {
                D->vid[dkey(d, x, y)] = nV;
                D->vx[nV] = x; D->vy[nV] = y; nV++;
            }
    D->nV = nV;
    if (nV != 2 * d * d + 2 * d + 1) return fail(OR_ERR_ASSERT, "|A<>| = %d", nV, 0);
    /* reflect every edge of T into the four quadrants; a set, so the copies
     * of axis edges that coincide are kept once */
    unsigned char *seen = calloc((size_t)nV * nV, 1);
    D->E = malloc(sizeof(int[2]) * 4 * T->n_edges);
    int nE = 0;
    static const int eps[4][2] = {{1, 1}, {-1, 1}, {1, -1}, {-1, -1}};
    for (int k = 0; k < T->n_edges; k++)
        for (int q = 0; q < 4; q++) {
            int u = D->vid[dkey(d, eps[q][0] * T->e[k][0], eps[q][1] * T->e[k][1])];
            int v = D->vid[dkey(d, eps[q][0] * T->e[k][2], eps[q][1] * T->e[k][3])];
            if (seen[u * nV + v]) continue;
            seen[u * nV + v] = seen[v * nV + u] = 1;
            D->E[nE][0] = u; D->E[nE][1] = v; nE++;
        }
    free(seen);
    D->nE = nE;
    if (nE != 6 * d * d + 2 * d) return fail(OR_ERR_ASSERT, "|E(T<>)| = %d, expected %d", nE, 6 * d * d + 2 * d);
    /* antipodal boundary pairs (i,d-i)~(-i,i-d) and (i,i-d)~(-i,d-i),
     * 0<=i<=d; the corner pairs occur in both families and are kept once */
    D->P = malloc(sizeof(int[2]) * (2 * d + 2));
    int nP = 0;
    for (int fam = 0; fam < 2; fam++)
        for (int i = 0; i <= d; i++) {
            int x = i, y = fam == 0 ? d - i : i - d;
            int a = D->vid[dkey(d, x, y)], b = D->vid[dkey(d, -x, -y)];
            int dup = 0;
            for (int t = 0; t < nP; t++)
                if ((D->P[t][0] == a && D->P[t][1] == b) || (D->P[t][0] == b && D->P[t][1] == a)) dup = 1;
            if (dup) continue;
            D->P[nP][0] = a; D->P[nP][1] = b; nP++;
        }
    D->nP = nP;
    if (nP != 2 * d) return fail(OR_ERR_ASSERT, "%d antipodal pairs, expected %d", nP, 2 * d);
    return OR_OK;
}

/* ---- canonical rooted-tree code (O9) ---- */

typedef struct {
    int n;
    int *parent;     /* -1 for the root */
} rtree_t;

static int cmp_desc(const void *a, const void *b) {
    return -strcmp(*(char *const *)a, *(char *const *)b);
}

/* '1' . sorted-descending children codes . '0' (caller frees) */
static char *ahu(const rtree_t *t, int v) {
    int nc = 0;
    for (int c = 0; c < t->n; c++) if (t->parent[c] == v) nc++;
    char **ch = malloc(sizeof(char *) * (nc + 1));
    int k = 0;
    size_t len = 2;
    for (int c = 0; c < t->n; c++)
        if (t->parent[c] == v) { ch[k] = ahu(t, c); len += strlen(ch[k]); k++; }
    qsort(ch, nc, sizeof(char *), cmp_desc);
    char *s = malloc(len + 1);
    s[0] = '1'; s[1] = 0;
    for (k = 0; k < nc; k++) { strcat(s, ch[k]); free(ch[k]); }
    strcat(s, "0");
    free(ch);
    return s;
}

/* W = concat of the root's children codes, sorted descending.  Returned
 * without the root's own parentheses. */
static char *scheme_word(const rtree_t *t, int root) {
    char *r = ahu(t, root);
    size_t L = strlen(r);
    char *w = malloc(L);
    memcpy(w, r + 1, L - 2);
    w[L - 2] = 0;
    free(r);
    return w;
}

/* code = 2^|W| + int(W), bit 127 for J */
static int word_to_code(const char *w, int odd, uint64_t code[2]) {
    size_t L = strlen(w);
    if (L + 1 > 127) return fail(OR_ERR_ASSERT, "scheme word of %d bits does not fit", (int)L, 0);
    code[0] = code[1] = 0;
    /* the bit string '1' . W, most significant first */
    size_t n = L + 1;
    for (size_t k = 0; k < n; k++) {
        int bit = k == 0 ? 1 : (w[k - 1] == '1');
        size_t pos = n - 1 - k;
        if (bit) code[pos / 64] |= (uint64_t)1 << (pos % 64);
    }
    if (odd) code[1] |= (uint64_t)1 << 63;
    return OR_OK;
}

/* ---- one evaluation of Algorithm 1 (O2-O9) ---- */

typedef struct {
    int n_components, n_regions, n_ovals, root, max_depth;
} info_t;

static int bfs_label(int n, const int *adj_start, const int *adj_list, int *label) {
    int *queue = malloc(sizeof(int) * (n > 0 ? n : 1));
    int nl = 0;
    for (int v = 0; v < n; v++) label[v] = -1;
    for (int s = 0; s < n; s++) {
        if (label[s] >= 0) continue;
        int h = 0, t = 0;
        queue[t++] = s; label[s] = nl;
        while (h < t) {
            int v = queue[h++];
            for (int k = adj_start[v]; k < adj_start[v + 1]; k++) {
                int u = adj_list[k];
                if (label[u] < 0) { label[u] = nl; queue[t++] = u; }
            }
        }
        nl++;
    }
    free(queue);
    return nl;
}

/* adjacency lists from an edge list (plain counting sort) */
static void make_adj(int n, int m, int (*E)[2], const unsigned char *keep, int *start, int *list) {
    for (int v = 0; v <= n; v++) start[v] = 0;
    for (int k = 0; k < m; k++)
        if (keep[k]) { start[E[k][0] + 1]++; start[E[k][1] + 1]++; }
    for (int v = 0; v < n; v++) start[v + 1] += start[v];
    int *fill = malloc(sizeof(int) * (n + 1));
    memcpy(fill, start, sizeof(int) * (n + 1));
    for (int k = 0; k < m; k++)
        if (keep[k]) { list[fill[E[k][0]]++] = E[k][1]; list[fill[E[k][1]]++] = E[k][0]; }
    free(fill);
}

static int evaluate(const diamond_t *D, const uint64_t mask[2], uint64_t code[2], info_t *info) {
    int d = D->d, nV = D->nV, nE = D->nE, nP = D->nP;
    int rc = OR_OK;
    /* O2: sigma on A from the mask, then eq. (signs) on A<> */
    int *sigma = malloc(sizeof(int) * D->nA);
    for (int k = 0; k < D->nA; k++) sigma[k] = (int)((mask[k / 64] >> (k % 64)) & 1);
    int *s = malloc(sizeof(int) * nV);
    for (int v = 0; v < nV; v++) {
        int x = D->vx[v], y = D->vy[v];
        int i = iabs(x), j = iabs(y);
        int sg = sigma[oracle_point_index(d, i, j)];
        if (x < 0) sg += i;          /* sigma(-i,j) = sigma(i,j) + i */
        if (y < 0) sg += j;          /* sigma(i,-j) = sigma(i,j) + j */
        s[v] = sg % 2;
    }
    /* O3: crossed edges */
    unsigned char *crossed = malloc(nE), *uncrossed = malloc(nE);
    for (int k = 0; k < nE; k++) {
        crossed[k] = s[D->E[k][0]] != s[D->E[k][1]];
        uncrossed[k] = !crossed[k];
    }
    /* O4: components of the subgraph of non-crossed edges */
    int *start = malloc(sizeof(int) * (nV + 1)), *list = malloc(sizeof(int) * 2 * nE);
    int *comp = malloc(sizeof(int) * nV);
    make_adj(nV, nE, D->E, uncrossed, start, list);
    int nC = bfs_label(nV, start, list, comp);
    /* O5: regions = components merged along antipodal pairs (both parities
     * of d: the pair is one point of RP^2 whatever the signs) */
    int (*CE)[2] = malloc(sizeof(int[2]) * (nP > 0 ? nP : 1));
    unsigned char *all = malloc(nP > 0 ? nP : 1);
    for (int t = 0; t < nP; t++) { CE[t][0] = comp[D->P[t][0]]; CE[t][1] = comp[D->P[t][1]]; all[t] = 1; }
    int *cstart = malloc(sizeof(int) * (nC + 1)), *clist = malloc(sizeof(int) * (2 * nP + 1));
    int *creg = malloc(sizeof(int) * nC);
    make_adj(nC, nP, CE, all, cstart, clist);
    int nR = bfs_label(nC, cstart, clist, creg);
    /* O6: region adjacency graph from crossed edges */
    unsigned char *pair = calloc((size_t)nR * nR, 1);
    unsigned char *selfloop = calloc(nR, 1);
    for (int k = 0; k < nE; k++) {
        if (!crossed[k]) continue;
        int a = creg[comp[D->E[k][0]]], b = creg[comp[D->E[k][1]]];
        if (a == b) selfloop[a] = 1;
        else pair[a * nR + b] = pair[b * nR + a] = 1;
    }
    /* O7: the root */
    int root = -1, nroot = 0;
    if (d % 2 == 1) {
        for (int r = 0; r < nR; r++) if (selfloop[r]) { root = r; nroot++; }
    } else {
        for (int r = 0; r < nR; r++)
            if (selfloop[r]) { rc = fail(OR_ERR_ASSERT, "self-loop at region %d for even d=%d", r, d); goto out; }
        /* two-colour the antipodal component multigraph; a conflict (a
         * self-loop included) is an odd cycle */
        int *col = malloc(sizeof(int) * nC);
        int *queue = malloc(sizeof(int) * nC);
        unsigned char *odd = calloc(nR, 1);
        for (int c = 0; c < nC; c++) col[c] = -1;
        for (int c0 = 0; c0 < nC; c0++) {
            if (col[c0] >= 0) continue;
            int h = 0, t = 0;
            queue[t++] = c0; col[c0] = 0;
            while (h < t) {
                int c = queue[h++];
                for (int k = cstart[c]; k < cstart[c + 1]; k++) {
                    int u = clist[k];
                    if (col[u] < 0) { col[u] = 1 - col[c]; queue[t++] = u; }
                    else if (col[u] == col[c]) odd[creg[c]] = 1;
                }
            }
        }
        for (int r = 0; r < nR; r++) if (odd[r]) { root = r; nroot++; }
        free(col); free(queue); free(odd);
    }
    if (nroot != 1) { rc = fail(OR_ERR_ASSERT, "%d root candidates (d=%d)", nroot, d); goto out; }
    /* O8: the adjacency graph is a tree; orient it away from the root */
    {
        int npairs = 0;
        for (int a = 0; a < nR; a++) for (int b = a + 1; b < nR; b++) npairs += pair[a * nR + b];
        if (npairs != nR - 1) { rc = fail(OR_ERR_ASSERT, "%d adjacency edges for %d regions", npairs, nR); goto out; }
        rtree_t t;
        t.n = nR;
        t.parent = malloc(sizeof(int) * nR);
        int *depth = malloc(sizeof(int) * nR), *queue = malloc(sizeof(int) * nR);
        for (int r = 0; r < nR; r++) depth[r] = -1;
        int h = 0, q = 0;
        queue[q++] = root; depth[root] = 0; t.parent[root] = -1;
        int maxdep = 0;
        while (h < q) {
            int a = queue[h++];
            for (int b = 0; b < nR; b++)
                if (pair[a * nR + b] && depth[b] < 0) {
                    depth[b] = depth[a] + 1; t.parent[b] = a; queue[q++] = b;
                    if (depth[b] > maxdep) maxdep = depth[b];
                }
        }
        if (q != nR) { free(t.parent); free(depth); free(queue); rc = fail(OR_ERR_ASSERT, "adjacency graph disconnected (%d of %d)", q, nR); goto out; }
        /* O9 */
        char *w = scheme_word(&t, root);
        rc = word_to_code(w, d % 2, code);
        free(w);
        if (info) {
            info->n_components = nC; info->n_regions = nR; info->n_ovals = nR - 1;
            info->root = root; info->max_depth = maxdep;
        }
        free(t.parent); free(depth); free(queue);
    }
out:
    free(sigma); free(s); free(crossed); free(uncrossed); free(start); free(list); free(comp);
    free(CE); free(all); free(cstart); free(clist); free(creg); free(pair); free(selfloop);
    return rc;
}

/* ---- exported entry points ---- */

int oracle_validate(int d, const int32_t *edges, int n_edges) {
    tri_t T;
    int rc = tri_build(d, edges, n_edges, &T);
    if (rc == OR_OK) tri_free(&T);
    return rc;
}

/* triangles of T (d^2 rows of 3 point indices); for the test-side checkers */
int oracle_triangles(int d, const int32_t *edges, int n_edges, int32_t *out_tri) {
    tri_t T;
    int rc = tri_build(d, edges, n_edges, &T);
    if (rc != OR_OK) return rc;
    for (int t = 0; t < T.n_tri; t++)
        for (int k = 0; k < 3; k++) out_tri[3 * t + k] = T.tri[t][k];
    tri_free(&T);
    return OR_OK;
}

/* diamond sizes: out[0]=|A<>|, out[1]=|E(T<>)|, out[2]=#antipodal pairs */
int oracle_diamond_sizes(int d, const int32_t *edges, int n_edges, int32_t out[3]) {
    tri_t T;
    diamond_t D;
    int rc = tri_build(d, edges, n_edges, &T);
    if (rc != OR_OK) return rc;
    rc = diamond_build(&T, &D);
    if (rc == OR_OK) { out[0] = D.nV; out[1] = D.nE; out[2] = D.nP; }
    diamond_free(&D);
    tri_free(&T);
    return rc;
}

/* one pair (T, sigma): code[2] and, if info != NULL, five counts
 * (components, regions, ovals, root region, max depth) */
int oracle_scheme(int d, const int32_t *edges, int n_edges, const uint64_t mask[2], uint64_t code[2], int32_t *info) {
    tri_t T;
    diamond_t D;
    int rc = tri_build(d, edges, n_edges, &T);
    if (rc != OR_OK) return rc;
    rc = diamond_build(&T, &D);
    if (rc == OR_OK) {
        info_t in;
        rc = evaluate(&D, mask, code, &in);
        if (rc == OR_OK && info) {
            info[0] = in.n_components; info[1] = in.n_regions; info[2] = in.n_ovals;
            info[3] = in.root; info[4] = in.max_depth;
        }
    }
    diamond_free(&D);
    tri_free(&T);
    return rc;
}

typedef struct {
    const diamond_t *D;
    const uint64_t *masks;
    uint64_t *codes;
    int64_t lo, hi;
    int rc;
    char err[256];
} job_t;

static void *worker(void *arg) {
    job_t *j = arg;
    j->rc = OR_OK;
    for (int64_t k = j->lo; k < j->hi; k++) {
        int rc = evaluate(j->D, j->masks + 2 * k, j->codes + 2 * k, NULL);
        if (rc != OR_OK) { j->rc = rc; memcpy(j->err, g_err, sizeof j->err); break; }
    }
    return NULL;
}

/* many masks for one triangulation (n x 2 words in, n x 2 words out), split
 * into contiguous chunks over n_threads POSIX threads */
int oracle_scheme_many(int d, const int32_t *edges, int n_edges, const uint64_t *masks, int64_t n,
                       uint64_t *codes, int n_threads) {
    if (n < 0 || n_threads < 1) return fail(OR_ERR_ARG, "bad n or thread count (%d)", n_threads, 0);
    tri_t T;
    diamond_t D;
    int rc = tri_build(d, edges, n_edges, &T);
    if (rc != OR_OK) return rc;
    rc = diamond_build(&T, &D);
    if (rc != OR_OK) { diamond_free(&D); tri_free(&T); return rc; }
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < n_threads; t++) {
        jobs[t].D = &D; jobs[t].masks = masks; jobs[t].codes = codes;
        jobs[t].lo = n * t / n_threads; jobs[t].hi = n * (t + 1) / n_threads;
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
    for (int t = 0; t < n_threads; t++)
        if (jobs[t].rc != OR_OK) { rc = jobs[t].rc; memcpy(g_err, jobs[t].err, sizeof g_err); break; }
    diamond_free(&D);
    tri_free(&T);
    return rc;
}

/* the extended sign distribution on A<> (eq. (signs)): one row x, y, s per
 * diamond vertex, |A<>| rows; for pinning the sign rule in tests */
int oracle_diamond_signs(int d, const int32_t *edges, int n_edges, const uint64_t mask[2], int32_t *out) {
    tri_t T;
    diamond_t D;
    int rc = tri_build(d, edges, n_edges, &T);
    if (rc != OR_OK) return rc;
    rc = diamond_build(&T, &D);
    if (rc == OR_OK) {
        for (int v = 0; v < D.nV; v++) {
            int x = D.vx[v], y = D.vy[v];
            int i = iabs(x), j = iabs(y);
            int k = oracle_point_index(d, i, j);
            int sg = (int)((mask[k / 64] >> (k % 64)) & 1);
            if (x < 0) sg += i;
            if (y < 0) sg += j;
            out[3 * v] = x; out[3 * v + 1] = y; out[3 * v + 2] = sg % 2;
        }
    }
    diamond_free(&D);
    tri_free(&T);
    return rc;
}
