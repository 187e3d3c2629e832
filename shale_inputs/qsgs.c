/*
 * Seeded quartet-structure-generation-set (QSGS) growth for synthetic shale
 * maps.  This is an input generator only: it decides which lattice nodes are
 * pore, inorganic matter (IOM) or organic matter (OM).  It holds none of the
 * lattice Boltzmann arithmetic and is shared, as an input, by the FP64 CPU
 * oracle and the GPU path.
 *
 * Growth rule (synchronous QSGS): every allowed node becomes a seed with
 * probability p_seed.  In each growth iteration a node that is not yet grown
 * becomes grown if at least one grown neighbour in direction d "fires", which
 * it does independently with probability p_d per iteration.  Because every
 * (grown node, direction, iteration) trial is independent, the iteration at
 * which a node is grown equals the first-passage time
 *     T(v) = min over neighbours u of  T(u) + W(u, d),
 * with W(u, d) ~ Geometric(p_d) on {1, 2, ...} drawn once per directed edge.
 * The map is therefore computed exactly with Dijkstra's algorithm instead of
 * thousands of sweeps.  Nodes are accepted in order of (T, random key) until
 * the target count is reached, which realises "stop at the first iteration that
 * reaches the target, accept the last iteration's nodes in random order".
 *
 * Random numbers: a counter-based generator, SplitMix64 (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to
 * (seed, stream, counter), so the map depends on the seed only, not on the
 * traversal order or thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t ctr)
{
    return mix64(mix64(seed ^ mix64(stream)) ^ ctr);
}

/* uniform in (0, 1] */
static inline double unit(uint64_t h) { return ((double)(h >> 11) + 1.0) * (1.0 / 9007199254740992.0); }

typedef struct { uint64_t key; uint32_t v; uint32_t pad; } hitem;

typedef struct { hitem* a; size_t n, cap; } heap_t;

static int heap_push(heap_t* h, uint64_t key, uint32_t v)
{
    if (h->n == h->cap) {
        size_t nc = h->cap ? h->cap * 2 : 1024;
        hitem* na = (hitem*)realloc(h->a, nc * sizeof(hitem));
        if (!na) return -1;
        h->a = na; h->cap = nc;
    }
    size_t i = h->n++;
    while (i > 0) {
        size_t p = (i - 1) / 2;
        if (h->a[p].key <= key) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].key = key; h->a[i].v = v; h->a[i].pad = 0;
    return 0;
}

static hitem heap_pop(heap_t* h)
{
    hitem top = h->a[0];
    hitem last = h->a[--h->n];
    size_t i = 0, n = h->n;
    for (;;) {
        size_t l = 2 * i + 1, r = l + 1, m = i;
        uint64_t km = last.key;
        if (l < n && h->a[l].key < km) { m = l; km = h->a[l].key; }
        if (r < n && h->a[r].key < km) { m = r; }
        if (m == i) break;
        h->a[i] = h->a[m];
        i = m;
    }
    if (n) h->a[i] = last;
    return top;
}

/*
 * Grow `target` nodes among those with allowed[v] != 0.
 *   nx, ny, nz      grid (x fastest); periodic neighbourhood
 *   ndir            number of neighbour offsets
 *   off             ndir * 3 integer offsets (dx, dy, dz)
 *   prob            ndir growth probabilities per iteration
 *   p_seed          seed probability per allowed node
 *   seed, stream    generator key
 *   out             nx*ny*nz bytes, set to 1 for grown nodes, 0 otherwise
 * Returns the number of grown nodes (== target unless fewer nodes are allowed
 * or reachable), or -1 on allocation failure.
 */
int64_t qsgs_grow(int32_t nx, int32_t ny, int32_t nz, int32_t ndir, const int32_t* off,
                  const double* prob, double p_seed, uint64_t seed, uint64_t stream,
                  const uint8_t* allowed, int64_t target, uint8_t* out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    memset(out, 0, (size_t)N);
    if (target <= 0) return 0;
    uint32_t* T = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    if (!T) return -1;
    for (int64_t v = 0; v < N; ++v) T[v] = UINT32_MAX;
    double lq[64];
    for (int d = 0; d < ndir && d < 64; ++d) lq[d] = log1p(-prob[d]);

    heap_t h = { 0, 0, 0 };
    const uint64_t s_seed = 4 * stream + 0, s_key = 4 * stream + 1, s_edge = 4 * stream + 2;
    for (int64_t v = 0; v < N; ++v) {
        if (!allowed[v]) continue;
        if (unit(draw(seed, s_seed, (uint64_t)v)) <= p_seed) {
            T[v] = 0;
            uint32_t rk = (uint32_t)(draw(seed, s_key, (uint64_t)v) >> 32);
            if (heap_push(&h, (uint64_t)rk, (uint32_t)v)) { free(T); free(h.a); return -1; }
        }
    }
    int64_t grown = 0;
    while (h.n && grown < target) {
        hitem it = heap_pop(&h);
        const uint32_t v = it.v;
        const uint32_t tv = (uint32_t)(it.key >> 32);
        if (out[v] || tv != T[v]) continue; /* stale entry */
        out[v] = 1;
        ++grown;
        const int32_t x = (int32_t)(v % (uint32_t)nx);
        const int32_t y = (int32_t)((v / (uint32_t)nx) % (uint32_t)ny);
        const int32_t z = (int32_t)(v / ((uint32_t)nx * (uint32_t)ny));
        for (int d = 0; d < ndir; ++d) {
            int32_t xx = (x + off[3 * d + 0] + nx) % nx;
            int32_t yy = (y + off[3 * d + 1] + ny) % ny;
            int32_t zz = (z + off[3 * d + 2] + nz) % nz;
            int64_t w = ((int64_t)zz * ny + yy) * nx + xx;
            if (!allowed[w] || out[w]) continue;
            /* Geometric waiting time on {1,2,...}: first iteration that fires. */
            double u = unit(draw(seed, s_edge, (uint64_t)v * 64u + (uint64_t)d));
            double wt = floor(log(u) / lq[d]) + 1.0;
            double tn = (double)tv + wt;
            if (tn >= 4.0e9) continue;
            uint32_t t32 = (uint32_t)tn;
            if (t32 < T[w]) {
                T[w] = t32;
                uint32_t rk = (uint32_t)(draw(seed, s_key, (uint64_t)w) >> 32);
                if (heap_push(&h, ((uint64_t)t32 << 32) | rk, (uint32_t)w)) { free(T); free(h.a); return -1; }
            }
        }
    }
    free(T);
    free(h.a);
    return grown;
}
