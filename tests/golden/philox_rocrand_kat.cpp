// Prints Philox4x32-10 outputs from rocRAND's host implementation for
// (key, counter) tuples read from stdin: "k0 k1 c0 c1 c2 c3" per line.
// Used by tests/test_oracle_rng.py as an external library reference; the
// engine's own ten-round function is called on the given counter and key.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct kat_engine : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};
int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    kat_engine eng;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        uint4 c; c.x = c0; c.y = c1; c.z = c2; c.w = c3;
        uint2 k; k.x = k0; k.y = k1;
        uint4 r = eng.run(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
