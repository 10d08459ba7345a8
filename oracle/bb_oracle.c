/*
 * bb_oracle.c -- plain, slow, sequential CPU oracle for the Barabasi-Albert
 * edge generator of Sanders & Schulz, "Scalable Generation of Scale-free
 * Graphs" (arXiv:1602.07106).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library under
 * paper_1602_07106_amd/ may include, link or call this file; only tests/,
 * __graft_entry__.smoke() and the cpu_baseline leg of bench.py use it.  It
 * shares no source, header, table or constant generator with the HIP path.
 *
 * What it computes (all arithmetic on unsigned 64-bit integers, mod 2^64):
 *
 *   key      = seed * 0x9E3779B97F4A7C15
 *   fmix64   = the SplitMix64 output mix (Steele, Lea & Flood, OOPSLA 2014)
 *   umul64hi = floor(a * b / 2^64)
 *   h(r)     = umul64hi(fmix64(r XOR key), r)        -- a value in 0..r-1
 *
 *   Batagelj-Brandes over an empty seed graph (paper Section 2):
 *     E[2i]   = floor(i / d)
 *     E[2i+1] = E[x], x = h(2i+1), x in 0..2i        for i = 0 .. n*d-1
 *
 *   Per-edge definition (paper Section 2, figure "generateEdge"): E[2i+1]
 *   follows the positions r = 2i+1, h(r), h(h(r)), ... (h applied at least
 *   once) until the first even position 2j, whose entry is floor(j/d).
 *
 *   Degrees: deg[v] = number of positions p in 0..2m-1 with E[p] = v, so a
 *   self-loop counts twice and the degrees sum to 2m.
 *
 *   Edge checksum word: w_i = (u_i * 2^32 + v_i) * (2i + 1)  mod 2^64; the
 *   checksum of a set of edges is the XOR of their words.
 */
#include <stdint.h>
#include <stddef.h>

#define BBO_PHI64 0x9E3779B97F4A7C15ull

/* Key of a graph: the seed times the 64-bit golden ratio, wrapping. */
uint64_t bbo_key(uint64_t seed) { return seed * BBO_PHI64; }

/* SplitMix64 output mix: three xor-shifts and two odd multiplies. */
uint64_t bbo_fmix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

/* High 64 bits of the full 128-bit product. */
uint64_t bbo_umul64hi(uint64_t a, uint64_t b)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    return (uint64_t)(p >> 64);
}

/* The keyed position hash: maps r >= 1 to a value in 0..r-1. */
uint64_t bbo_h(uint64_t key, uint64_t r) { return bbo_umul64hi(bbo_fmix64(r ^ key), r); }

/* Checksum word of edge i = (u, v). */
uint64_t bbo_edge_word(uint64_t i, uint64_t u, uint64_t v)
{
    return ((u << 32) + v) * (2 * i + 1);
}

/*
 * Sequential Batagelj-Brandes (paper Section 2) with the keyed hash as the
 * source of the choice x in 0..2i.  Fills E[0 .. 2*n*d-1].  Node IDs must fit
 * 32 bits.  Returns 0, -1 for arguments it cannot hold, or -2 if the hash
 * ever leaves 0..2i (which the hash definition rules out).
 */
int bbo_bb_generate(uint64_t n, uint64_t d, uint64_t seed, uint32_t *E, uint64_t *hash_calls)
{
    if (n > 0xFFFFFFFFull) return -1;
    uint64_t m = n * d;
    uint64_t key = bbo_key(seed);
    for (uint64_t i = 0; i < m; i++) {
        E[2 * i] = (uint32_t)(i / d);
        uint64_t x = bbo_h(key, 2 * i + 1);
        if (x > 2 * i) return -2;
        E[2 * i + 1] = E[x];
    }
    if (hash_calls) *hash_calls = m;
    return 0;
}

/*
 * Sequential Batagelj-Brandes with the choices given explicitly:
 * x[i] must lie in 0..2i.  Used to check the model itself on tiny inputs.
 * Returns 0, or -1 when some x[i] is out of range.
 */
int bbo_bb_with_choices(uint64_t n, uint64_t d, const uint64_t *x, uint32_t *E)
{
    uint64_t m = n * d;
    for (uint64_t i = 0; i < m; i++) {
        if (x[i] > 2 * i) return -1;
        E[2 * i] = (uint32_t)(i / d);
        E[2 * i + 1] = E[x[i]];
    }
    return 0;
}

/*
 * deg[v] = occurrences of v among E[0 .. len-1]; deg has n entries.  Returns
 * 0, or -1 if some entry is not a node ID below n.
 */
int bbo_count_degrees(const uint32_t *E, uint64_t len, uint64_t n, uint64_t *deg)
{
    for (uint64_t v = 0; v < n; v++) deg[v] = 0;
    for (uint64_t p = 0; p < len; p++) {
        if (E[p] >= n) return -1;
        deg[E[p]] += 1;
    }
    return 0;
}

/* XOR of the checksum words of the m edges stored in E. */
uint64_t bbo_checksum_E(const uint32_t *E, uint64_t m)
{
    uint64_t cs = 0;
    for (uint64_t i = 0; i < m; i++) cs ^= bbo_edge_word(i, E[2 * i], E[2 * i + 1]);
    return cs;
}

/*
 * Edge i from the definition of E alone: the first endpoint is floor(i/d);
 * the second is E[2i+1], found by following h from position 2i+1 (at least
 * one step) until the position is even.  *steps receives the number of hash
 * evaluations.
 */
void bbo_edge(uint64_t d, uint64_t seed, uint64_t i, uint64_t *u, uint64_t *v, uint64_t *steps)
{
    uint64_t key = bbo_key(seed);
    uint64_t r = 2 * i + 1;
    uint64_t k = 0;
    do {
        r = bbo_h(key, r);
        k++;
    } while (r & 1);
    *u = i / d;
    *v = r / (2 * d);
    if (steps) *steps = k;
}

/* Edges i0 .. i0+count-1, one at a time: out[2j] = u, out[2j+1] = v. */
void bbo_edges_range(uint64_t d, uint64_t seed, uint64_t i0, uint64_t count, uint64_t *out,
                     uint64_t *hash_calls)
{
    uint64_t total = 0;
    for (uint64_t j = 0; j < count; j++) {
        uint64_t u, v, k;
        bbo_edge(d, seed, i0 + j, &u, &v, &k);
        out[2 * j] = u;
        out[2 * j + 1] = v;
        total += k;
    }
    if (hash_calls) *hash_calls = total;
}

/*
 * Streaming consumer over edges i0 .. i0+count-1 (paper Section 3): adds the
 * number of endpoints equal to v to deg_k[v] for every v < k, and XORs the
 * checksum words of the edges into *cs.  Nothing is stored.
 */
void bbo_stream(uint64_t d, uint64_t seed, uint64_t i0, uint64_t count, uint64_t k,
                uint64_t *deg_k, uint64_t *cs, uint64_t *hash_calls)
{
    uint64_t total = 0;
    uint64_t x = 0;
    for (uint64_t j = 0; j < count; j++) {
        uint64_t i = i0 + j;
        uint64_t u, v, s;
        bbo_edge(d, seed, i, &u, &v, &s);
        if (u < k) deg_k[u] += 1;
        if (v < k) deg_k[v] += 1;
        x ^= bbo_edge_word(i, u, v);
        total += s;
    }
    *cs ^= x;
    if (hash_calls) *hash_calls = total;
}
