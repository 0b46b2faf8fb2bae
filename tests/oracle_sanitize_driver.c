/*
 * Driver that runs the CPU oracle (oracle/rsea_oracle.c) under AddressSanitizer
 * and UndefinedBehaviorSanitizer.  Test infrastructure: it is compiled and run
 * by tests/test_oracle_sanitized.py only.
 *
 * Input file (little-endian):
 *   u32 q, r, delta, eta, k, theta, key_bits, verify_rehash, n_routers, n_slices
 *   u32 tables[2][4][256]
 *   per slice: u64 n, then u32 pairs[n][2]
 * Every slice's pairs are dealt round-robin to n_routers router detectors and
 * also scanned by one detector that sees them all; each slot the routers are
 * merged into a global detector (Alg. 5) and both the global and the union
 * detector reconstruct; routers only age.  Every other oracle entry point is
 * exercised too.  Output, per slice: "slice t n" and n lines "ip rk est" of
 * the union detector's list, then "merged-equal 0|1".
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_rsea orc_rsea;
orc_rsea *orc_create(uint32_t q, uint32_t r, uint32_t delta, uint32_t eta, uint32_t k, uint32_t theta,
                     uint32_t key_bits, uint32_t verify_rehash, const uint32_t *tables);
void orc_destroy(orc_rsea *s);
void orc_scan(orc_rsea *s, const uint32_t *pairs, uint64_t n);
int64_t orc_close(orc_rsea *s, int advance_only);
uint64_t orc_results(const orc_rsea *s, uint32_t *ip, uint32_t *rk, double *est, uint64_t cap);
void orc_rk(const orc_rsea *s, uint32_t *out);
void orc_hse(const orc_rsea *s, uint32_t *counts, uint32_t *out);
uint64_t orc_tuples(const orc_rsea *s, uint32_t *out, uint64_t cap);
void orc_canonical(const orc_rsea *s, uint16_t *out);
int orc_merge(orc_rsea *g, orc_rsea *const *routers, uint32_t n);
uint64_t orc_roundtrip_failures(const orc_rsea *s, uint64_t lo, uint64_t hi, uint64_t stride);
uint64_t orc_extract(const orc_rsea *s, const uint32_t *ct);
uint64_t orc_bruteforce(const orc_rsea *s, uint64_t x_lo, uint64_t x_hi, uint32_t *ip, uint32_t *rk, uint64_t cap);
int64_t orc_reconstruct(orc_rsea *s);
void orc_age(orc_rsea *s);
uint32_t orc_h1(const orc_rsea *s, uint32_t oip);
void orc_rhfg(const orc_rsea *s, uint32_t cip, uint32_t *cols);

static void need(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "driver: %s\n", what);
        exit(2);
    }
}

int main(int argc, char **argv)
{
    need(argc == 2, "usage: driver input.bin");
    FILE *f = fopen(argv[1], "rb");
    need(f != NULL, "cannot open input");
    uint32_t hdr[10];
    need(fread(hdr, 4, 10, f) == 10, "short header");
    const uint32_t q = hdr[0], r = hdr[1], delta = hdr[2], eta = hdr[3], k = hdr[4], theta = hdr[5];
    const uint32_t key_bits = hdr[6], rehash = hdr[7], n_routers = hdr[8], n_slices = hdr[9];
    need(n_routers >= 1 && n_routers <= 16, "router count");
    uint32_t *tables = malloc(2048 * 4);
    need(tables && fread(tables, 4, 2048, f) == 2048, "short tables");
    orc_rsea *uni = orc_create(q, r, delta, eta, k, theta, key_bits, rehash, tables);
    orc_rsea *glob = orc_create(q, r, delta, eta, k, theta, key_bits, rehash, tables);
    orc_rsea *rt[16];
    for (uint32_t j = 0; j < n_routers; j++) {
        rt[j] = orc_create(q, r, delta, eta, k, theta, key_bits, rehash, tables);
        need(rt[j] != NULL, "router create");
    }
    need(uni && glob, "create");
    const uint64_t n_se = (uint64_t)r << q, n_cells = n_se * eta;
    uint16_t *ca = malloc(n_cells * 2), *cb = malloc(n_cells * 2);
    uint32_t *rka = malloc(n_se * 4), *rkb = malloc(n_se * 4);
    uint32_t *hc = malloc(r * 4), *hl = malloc(n_se * 4);
    need(ca && cb && rka && rkb && hc && hl, "alloc");
    for (uint32_t t = 0; t < n_slices; t++) {
        uint64_t n = 0;
        need(fread(&n, 8, 1, f) == 1, "short slice header");
        uint32_t *pairs = malloc((n ? n : 1) * 8);
        need(pairs && fread(pairs, 8, n, f) == n, "short slice");
        orc_scan(uni, pairs, n);
        /* deal the pairs round-robin to the routers */
        for (uint32_t j = 0; j < n_routers; j++) {
            uint64_t m = 0;
            uint32_t *part = malloc((n / n_routers + 1) * 8);
            need(part != NULL, "alloc part");
            for (uint64_t i = j; i < n; i += n_routers, m++) {
                part[2 * m] = pairs[2 * i];
                part[2 * m + 1] = pairs[2 * i + 1];
            }
            orc_scan(rt[j], part, m);
            free(part);
        }
        free(pairs);
        need(orc_merge(glob, rt, n_routers) == 0, "merge");
        orc_canonical(uni, ca);
        orc_canonical(glob, cb);
        int equal = memcmp(ca, cb, n_cells * 2) == 0;
        need(orc_reconstruct(uni) >= 0 && orc_reconstruct(glob) >= 0, "reconstruct");
        orc_rk(uni, rka);
        orc_rk(glob, rkb);
        equal &= memcmp(rka, rkb, n_se * 4) == 0;
        orc_hse(uni, hc, hl);
        uint64_t nt = orc_tuples(uni, NULL, 0);
        uint32_t *tu = malloc((nt ? nt : 1) * r * 4);
        need(tu != NULL, "alloc tuples");
        orc_tuples(uni, tu, nt);
        for (uint64_t i = 0; i < nt && i < 64; i++) (void)orc_extract(uni, tu + i * r);
        free(tu);
        uint64_t m = orc_results(uni, NULL, NULL, NULL, 0);
        uint32_t *ip = malloc((m ? m : 1) * 4), *rk = malloc((m ? m : 1) * 4);
        double *est = malloc((m ? m : 1) * 8);
        need(ip && rk && est, "alloc results");
        orc_results(uni, ip, rk, est, m);
        uint64_t mg = orc_results(glob, NULL, NULL, NULL, 0);
        equal &= mg == m;
        printf("slice %u %llu\n", t, (unsigned long long)m);
        for (uint64_t i = 0; i < m; i++) printf("%u %u %.17g\n", ip[i], rk[i], est[i]);
        printf("merged-equal %d\n", equal);
        free(ip);
        free(rk);
        free(est);
        if (key_bits <= 16) {
            uint64_t nb = orc_bruteforce(uni, 0, 1ull << key_bits, NULL, NULL, 0);
            need(nb != UINT64_MAX, "bruteforce");
        }
        orc_age(uni);
        orc_age(glob);
        for (uint32_t j = 0; j < n_routers; j++) (void)orc_close(rt[j], 1);
    }
    uint32_t cols[64];
    orc_rhfg(uni, 0xC0A80001u, cols);
    (void)orc_h1(uni, 0x08080808u);
    need(orc_roundtrip_failures(uni, 0, 1ull << key_bits, key_bits > 16 ? 1000003 : 1) == 0, "roundtrip");
    free(ca);
    free(cb);
    free(rka);
    free(rkb);
    free(hc);
    free(hl);
    free(tables);
    for (uint32_t j = 0; j < n_routers; j++) orc_destroy(rt[j]);
    orc_destroy(uni);
    orc_destroy(glob);
    fclose(f);
    return 0;
}
