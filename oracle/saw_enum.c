/*
 * saw_enum.c -- brute-force count of self-avoiding walks, c_n.
 *
 * TEST INFRASTRUCTURE ONLY.  An exact enumeration used to pin the oracle's
 * free-neighbour scan and weight update against the quantity the Rosenbluth
 * counting theorem (Sec. 1, eqn (3)) says their expectation equals: c_n, the
 * number of n-step self-avoiding walks from the origin of Z^d.
 *
 * Depth-first search over a dense occupancy grid (side 2*n_max + 3, so a walk
 * never reaches the border).  It shares nothing with the oracle's hash set or
 * scan.  The lattice symmetry that maps any first step to +x is used: every
 * walk with n >= 1 is counted once with first step +x and the total is
 * multiplied by 2d.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int dim;
    int n_max;
    int64_t side;
    int64_t stride[3];
    uint8_t* grid;
    uint64_t* count;
    uint64_t* r2;        /* sum over walks of the squared end-to-end distance, or NULL */
    int64_t origin;
} saw_ctx;

static uint64_t saw_r2_of(const saw_ctx* c, int64_t pos)
{
    /* coordinates from the grid index (each in [0, side), the origin at n_max + 1) */
    uint64_t r2 = 0;
    int64_t rest = pos;
    for (int i = c->dim - 1; i >= 0; --i) {
        const int64_t coord = rest / c->stride[i] - (c->n_max + 1);
        rest %= c->stride[i];
        r2 += (uint64_t)(coord * coord);
    }
    return r2;
}

static void saw_dfs(saw_ctx* c, int64_t pos, int n)
{
    c->count[n] += 1;
    if (c->r2) c->r2[n] += saw_r2_of(c, pos);
    if (n == c->n_max) return;
    for (int axis = 0; axis < c->dim; ++axis) {
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            int64_t q = pos + sgn * c->stride[axis];
            if (!c->grid[q]) {
                c->grid[q] = 1;
                saw_dfs(c, q, n + 1);
                c->grid[q] = 0;
            }
        }
    }
}

/* count[n] = c_n for n = 0..n_max, and (r2 != NULL) r2[n] = the sum over
 * those walks of the squared end-to-end distance.  Returns 0 on success. */
int saw_count_r2(int dim, int n_max, uint64_t* count, uint64_t* r2)
{
    if (dim < 1 || dim > 3 || n_max < 0) return -1;
    saw_ctx c;
    c.dim = dim;
    c.n_max = n_max;
    c.side = 2 * (int64_t)n_max + 3;
    c.stride[0] = 1;
    c.stride[1] = c.side;
    c.stride[2] = c.side * c.side;
    int64_t cells = 1;
    for (int i = 0; i < dim; ++i) cells *= c.side;
    c.grid = (uint8_t*)calloc((size_t)cells, 1);
    if (!c.grid) return -1;
    uint64_t* half = (uint64_t*)calloc((size_t)n_max + 1, sizeof(uint64_t));
    if (!half) { free(c.grid); return -1; }
    c.count = half;
    uint64_t* half_r2 = NULL;
    if (r2) {
        half_r2 = (uint64_t*)calloc((size_t)n_max + 1, sizeof(uint64_t));
        if (!half_r2) { free(half); free(c.grid); return -1; }
    }
    c.r2 = half_r2;
    int64_t origin = 0;
    for (int i = 0; i < dim; ++i) origin += (int64_t)(n_max + 1) * c.stride[i];
    c.grid[origin] = 1;
    memset(count, 0, sizeof(uint64_t) * ((size_t)n_max + 1));
    count[0] = 1;
    if (n_max >= 1) {
        int64_t first = origin + 1;   /* first step +x */
        c.grid[first] = 1;
        saw_dfs(&c, first, 1);
        for (int n = 1; n <= n_max; ++n) count[n] = half[n] * (uint64_t)(2 * dim);
        /* rotations and reflections keep |end|^2, so the first-step symmetry holds for it too */
        if (r2)
            for (int n = 1; n <= n_max; ++n) r2[n] = half_r2[n] * (uint64_t)(2 * dim);
    }
    if (r2) r2[0] = 0;
    free(half_r2);
    free(half);
    free(c.grid);
    return 0;
}

int saw_count(int dim, int n_max, uint64_t* count) { return saw_count_r2(dim, n_max, count, NULL); }
