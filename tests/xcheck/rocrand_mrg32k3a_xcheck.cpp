// Independent cross-check of the oracle's MRG32k3a states: drives the
// open-source rocRAND MRG32k3a engine (header only, host side) from a given
// 6-word state.  Test infrastructure; never part of the product library.
//
// stdin, one query per line:  s0 s1 s2 s3 s4 s5 op k
//   op = step : print k outputs (integers in [1, m1]), then the state
//   op = skip : advance k steps, print the state
//   op = sub  : advance k substreams (2^76 steps each), print the state
//   op = seq  : advance k sequences (2^127 steps each), print the state
#include <rocrand/rocrand_mrg32k3a.h>

#include <cstdio>
#include <cstring>

struct Probe : rocrand_device::mrg32k3a_engine {
    void set(const unsigned s[6]) {
        for (int i = 0; i < 3; ++i) { m_state.g1[i] = s[i]; m_state.g2[i] = s[3 + i]; }
    }
    void print_state() {
        std::printf("%u %u %u %u %u %u\n", m_state.g1[0], m_state.g1[1], m_state.g1[2],
                    m_state.g2[0], m_state.g2[1], m_state.g2[2]);
    }
};

int main() {
    unsigned s[6];
    char op[16];
    unsigned long long k;
    while (std::scanf("%u %u %u %u %u %u %15s %llu", &s[0], &s[1], &s[2], &s[3], &s[4], &s[5],
                      op, &k) == 8) {
        Probe p;
        p.set(s);
        if (!std::strcmp(op, "step")) {
            for (unsigned long long i = 0; i < k; ++i) std::printf("%u ", p.next());
            std::printf("\n");
        } else if (!std::strcmp(op, "skip")) {
            p.discard(k);
        } else if (!std::strcmp(op, "sub")) {
            p.discard_subsequence(k);
        } else if (!std::strcmp(op, "seq")) {
            p.discard_sequence(k);
        } else {
            return 2;
        }
        p.print_state();
        std::fflush(stdout);
    }
    return 0;
}
