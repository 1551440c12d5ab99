/* Exercises the C oracle under AddressSanitizer/UndefinedBehaviorSanitizer:
   seeding, every request kind on several threads, the x-part stepping,
   Berlekamp-Massey, the primitivity test on a small trinomial, polynomial
   jump-ahead against plain stepping.  Exit status 0 and "OK" when every
   check holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t w, r, s, a, b, c, d, gamma;
    uint32_t omega;
} xgo_params;

int xgo_seed_streams(const xgo_params *p, uint64_t seed, uint64_t first, uint64_t count,
                     uint32_t *ring, uint32_t *weyl, uint64_t *pos);
int xgo_run_streams(const xgo_params *p, uint32_t *ring, uint32_t *weyl, uint64_t *pos,
                    uint64_t count, int kind, uint64_t n, void *out, uint64_t out_stride_bytes,
                    int threads);
int xgo_xpart_run(const xgo_params *p, uint32_t *ring, uint64_t steps, uint32_t bit,
                  uint8_t *bits_out);
int xgo_xpart_jump_poly(const xgo_params *p, uint32_t *ring, const uint64_t *g);
int gf2_berlekamp_massey(const uint8_t *bits, int N, uint64_t *poly, int words);
int gf2_is_primitive(const uint64_t *P, int n, const int *sub_exps, int nsub,
                     const uint64_t *exps, int nq, int exp_words);
int gf2_z_pow_mod(const uint64_t *P, int n, const uint8_t *jbits, int nbits, uint64_t *g);

#define CHECK(c) do { if (!(c)) { printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); return 1; } } while (0)

int main(void)
{
    const xgo_params P = {32, 128, 65, 15, 14, 12, 17, 16, 0x9E3779B9u};
    enum { S = 5 };
    uint32_t ring[S * 128], weyl[S];
    uint64_t pos[S];
    CHECK(xgo_seed_streams(&P, 42, 0, S, ring, weyl, pos) == 0);
    /* every kind, odd lengths, 3 threads over 5 streams */
    {
        const uint64_t n = 1001;
        void *out = malloc(S * n * 8 + 64);
        CHECK(out != NULL);
        for (int kind = 0; kind <= 4; ++kind)
            CHECK(xgo_run_streams(&P, ring, weyl, pos, S, kind, n, kind == 4 ? NULL : out,
                                  kind == 3 ? 3 * 8 : n * 8, 3) == 0);
        CHECK(xgo_run_streams(&P, ring, weyl, pos, S, 7, n, out, n * 8, 1) == -1);
        free(out);
    }
    /* the x-part's minimal polynomial has degree 4096 */
    enum { NB = 2 * 4096 + 64, PW = 65 };
    uint8_t *bits = malloc(NB);
    uint64_t poly[PW];
    uint32_t r0[128], r1[128];
    CHECK(bits != NULL);
    memcpy(r0, ring, sizeof(r0));
    CHECK(xgo_xpart_run(&P, r0, NB, 0, bits) == 0);
    CHECK(gf2_berlekamp_massey(bits, NB, poly, PW) == 4096);
    /* x^3 + x + 1 is primitive: n = 3 (prime), 2^3 - 1 = 7 (prime) */
    {
        const uint64_t tri = 0xB, one = 1;
        const int sub = 1;
        CHECK(gf2_is_primitive(&tri, 3, &sub, 1, &one, 1, 1) == 0);
    }
    /* jump by J = 1000 + 4096 with z^J mod P equals stepping */
    {
        const uint32_t J = 5096;
        uint8_t jb[13];
        uint64_t g[64];
        for (int i = 0; i < 13; ++i) jb[i] = (J >> i) & 1u;
        CHECK(gf2_z_pow_mod(poly, 4096, jb, 13, g) == 0);
        memcpy(r0, ring + 128, sizeof(r0));
        memcpy(r1, ring + 128, sizeof(r1));
        CHECK(xgo_xpart_run(&P, r0, J, 0, NULL) == 0);
        CHECK(xgo_xpart_jump_poly(&P, r1, g) == 0);
        CHECK(memcmp(r0, r1, sizeof(r0)) == 0);
    }
    free(bits);
    printf("OK\n");
    return 0;
}
