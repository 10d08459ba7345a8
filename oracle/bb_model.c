/*
 * bb_model.c -- oracle for the generalizations of the Barabasi-Albert
 * generator (Sanders & Schulz, arXiv:1602.07106, Section "Generalizations")
 * and for the paper's own CRC-based hash (figure with hash_crc).
 *
 * TEST INFRASTRUCTURE ONLY, like bb_oracle.c (built into the same library).
 *
 * The model.  A seed graph of n0 nodes and m0 edges occupies positions
 * 0 .. 2*m0-1 of the edge array E (S, given).  New nodes n0 .. n-1 each add
 * d edges; new edge i (i = 0 .. (n-n0)*d - 1) sits at positions P = 2*m0 +
 * 2i (first endpoint) and P+1:
 *
 *   E[P]   = n0 + floor(i/d)
 *   E[P+1] = E[x],  x drawn from 0 .. b-1 with
 *            b = P+1                      (self-loops allowed: every earlier
 *                                          position, as in the plain model)
 *            b = 2*m0 + 2*d*floor(i/d)    (no self-loops: only positions
 *                                          before the first edge of the new
 *                                          node, so it cannot pick itself)
 *
 * The draw at position r is a hash of r itself reduced into 0..b-1, so
 * each edge draws independently even when its bound is shared with the
 * other d-1 edges of its node.  Per-edge recomputation follows positions
 * r = P+1, x(r), x(x(r)), ... (at least one draw) until r < 2*m0 (a seed
 * position: node S[r]) or r is even (node n0 + floor((r - 2*m0) / (2d))).
 * With n0 = m0 = 0 and self-loops allowed this is the plain model of
 * bb_oracle.c exactly.
 *
 * Hashes of position r with key k = seed * phi64 into 0..b-1:
 *   fmix:  umul64hi(fmix64(r XOR k), b)
 *   crc:   ((crc32c(0, z) << 32) + crc32c(1, z)) mod b,  z = r XOR k
 * where crc32c(c, z) is the CRC-32C register update over the 8 bytes of z
 * (least significant first) from register value c, with no inversion: the
 * SSE4.2 crc32 instruction the paper's hash_crc uses.  With key 0 and
 * b = r the crc hash is the paper's hash_crc(r).
 */
#include <stdint.h>
#include <string.h>

uint64_t bbo_key(uint64_t seed);
uint64_t bbo_fmix64(uint64_t z);
uint64_t bbo_umul64hi(uint64_t a, uint64_t b);

enum { BBO_NO_LOOPS = 1, BBO_CRC = 2 };

/* CRC-32C register update over len bytes, one bit at a time (reflected
 * polynomial 0x82F63B78, no initial or final inversion). */
uint32_t bbo_crc32c_update(uint32_t crc, const unsigned char *p, uint64_t len)
{
    for (uint64_t k = 0; k < len; k++) {
        crc ^= p[k];
        for (int b = 0; b < 8; b++)
            crc = (crc >> 1) ^ (0x82F63B78u & (0u - (crc & 1u)));
    }
    return crc;
}

/* Update over the 8 bytes of x, least significant byte first. */
uint32_t bbo_crc32c_u64(uint32_t crc, uint64_t x)
{
    unsigned char b[8];
    for (int k = 0; k < 8; k++) b[k] = (unsigned char)(x >> (8 * k));
    return bbo_crc32c_update(crc, b, 8);
}

uint64_t bbo_h_crc(uint64_t key, uint64_t r, uint64_t bound)
{
    const uint64_t z = r ^ key;
    const uint64_t hash = ((uint64_t)bbo_crc32c_u64(0, z) << 32) + (uint64_t)bbo_crc32c_u64(1, z);
    return hash % bound;
}

uint64_t bbo_h_fmix(uint64_t key, uint64_t r, uint64_t bound) { return bbo_umul64hi(bbo_fmix64(r ^ key), bound); }

typedef struct {
    uint64_t n0, m0, n, d, key;
    const uint32_t *S;
    unsigned flags;
} Model;

/* Draw bound of the new edge whose second endpoint sits at odd r >= 2*m0. */
static uint64_t model_bound(const Model *M, uint64_t r)
{
    if (!(M->flags & BBO_NO_LOOPS)) return r;
    const uint64_t i = (r - 2 * M->m0 - 1) / 2;
    return 2 * M->m0 + 2 * M->d * (i / M->d);
}

static uint64_t model_draw(const Model *M, uint64_t r)
{
    const uint64_t b = model_bound(M, r);
    return (M->flags & BBO_CRC) ? bbo_h_crc(M->key, r, b) : bbo_h_fmix(M->key, r, b);
}

/* Arguments the model accepts: n0 <= n, node IDs fit 32 bits, positions fit
 * 64 bits, and without self-loops a non-empty seed graph (node n0 needs an
 * earlier position to attach to).  0 when valid, -1 otherwise. */
static int model_check(uint64_t n0, uint64_t m0, uint64_t n, uint64_t d, unsigned flags)
{
    if (n0 > n || n > ((uint64_t)1 << 32) || d == 0) return -1;
    if ((flags & BBO_NO_LOOPS) && m0 == 0 && n > n0) return -1;
    const unsigned __int128 pos = (unsigned __int128)2 * m0 + (unsigned __int128)2 * (n - n0) * d;
    if (pos >> 63) return -1;
    return 0;
}

/*
 * Sequential Batagelj-Brandes with the seed graph S (2*m0 node IDs) and the
 * hash as the source of the draws.  E receives all 2*m0 + 2*(n-n0)*d
 * positions.  Returns 0, -1 for arguments outside the model, -2 if a draw
 * ever leaves 0..b-1 (which the hash definitions rule out).
 */
int bbo_model_bb_generate(uint64_t n0, uint64_t m0, const uint32_t *S, uint64_t n, uint64_t d, uint64_t seed,
                          unsigned flags, uint32_t *E, uint64_t *hash_calls)
{
    if (model_check(n0, m0, n, d, flags)) return -1;
    const Model M = {n0, m0, n, d, bbo_key(seed), S, flags};
    for (uint64_t p = 0; p < 2 * m0; p++) E[p] = S[p];
    const uint64_t m = (n - n0) * d;
    for (uint64_t i = 0; i < m; i++) {
        const uint64_t P = 2 * m0 + 2 * i;
        E[P] = (uint32_t)(n0 + i / d);
        const uint64_t b = model_bound(&M, P + 1);
        const uint64_t x = model_draw(&M, P + 1);
        if (x >= b) return -2;
        E[P + 1] = E[x];
    }
    if (hash_calls) *hash_calls = m;
    return 0;
}

/* The same with the draws given: x[i] in 0 .. b_i - 1.  Returns 0, -1 for
 * arguments outside the model or a draw out of range. */
int bbo_model_bb_with_choices(uint64_t n0, uint64_t m0, const uint32_t *S, uint64_t n, uint64_t d, unsigned flags,
                              const uint64_t *x, uint32_t *E)
{
    if (model_check(n0, m0, n, d, flags)) return -1;
    const Model M = {n0, m0, n, d, 0, S, flags};
    for (uint64_t p = 0; p < 2 * m0; p++) E[p] = S[p];
    const uint64_t m = (n - n0) * d;
    for (uint64_t i = 0; i < m; i++) {
        const uint64_t P = 2 * m0 + 2 * i;
        E[P] = (uint32_t)(n0 + i / d);
        if (x[i] >= model_bound(&M, P + 1)) return -1;
        E[P + 1] = E[x[i]];
    }
    return 0;
}

/* Node held by a position where a chain ends. */
static uint32_t model_node(const Model *M, uint64_t r)
{
    if (r < 2 * M->m0) return M->S[r];
    return (uint32_t)(M->n0 + (r - 2 * M->m0) / (2 * M->d));
}

/*
 * Per-edge recomputation of new edge i: (u, v) and the number of draws.
 * With x given (non-NULL), the draw at odd position r >= 2*m0 is
 * x[(r - 2*m0 - 1) / 2] instead of the hash.
 */
void bbo_model_edge(uint64_t n0, uint64_t m0, const uint32_t *S, uint64_t d, uint64_t seed, unsigned flags,
                    const uint64_t *x, uint64_t i, uint64_t *u, uint64_t *v, uint64_t *steps)
{
    const Model M = {n0, m0, 0, d, bbo_key(seed), S, flags};
    uint64_t r = 2 * m0 + 2 * i + 1, s = 0;
    do {
        r = x ? x[(r - 2 * m0 - 1) / 2] : model_draw(&M, r);
        s++;
    } while (r >= 2 * m0 && (r & 1));
    *u = n0 + i / d;
    *v = model_node(&M, r);
    *steps = s;
}

/* New edges i0 .. i0+count-1 into out (pairs, uint32), total draws. */
void bbo_model_edges_range(uint64_t n0, uint64_t m0, const uint32_t *S, uint64_t d, uint64_t seed, unsigned flags,
                           uint64_t i0, uint64_t count, uint32_t *out, uint64_t *steps)
{
    uint64_t tot = 0;
    for (uint64_t k = 0; k < count; k++) {
        uint64_t u, v, s;
        bbo_model_edge(n0, m0, S, d, seed, flags, 0, i0 + k, &u, &v, &s);
        out[2 * k] = (uint32_t)u;
        out[2 * k + 1] = (uint32_t)v;
        tot += s;
    }
    *steps = tot;
}
