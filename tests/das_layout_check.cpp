// CPU check of the DAS LDS layout (das_layout.h), built with the host
// compiler by test_das_layout.py.  Exit status 0 when every check holds;
// otherwise prints the failed check and exits 1.
#include <cstdio>
#include <initializer_list>

#include "das_layout.h"

using wf::das_lds;
using wf::das_lds_fits;

static int failures = 0;

static void expect(bool ok, const char* what, int nbuf, int slot, int T) {
    if (!ok) {
        std::printf("FAIL %s (nbuf %d, slot %d, T %d)\n", what, nbuf, slot, T);
        ++failures;
    }
}

int main() {
    const int slots[] = {18, 34, 146, 274, 290, 514};
    const int Ts[] = {1, 5, 64, 128, 1024};
    for (int nbuf : {2, 4}) {
        for (int slot : slots) {
            for (int T : Ts) {
                const wf::DasLds L = das_lds(nbuf, slot, T);
                const size_t win = (size_t)nbuf * wf::kChunk * slot * 8;
                expect(L.m_tab == win, "tables follow the window arrays", nbuf, slot, T);
                expect(L.m_tab % 16 == 0 && L.q_tab % 16 == 0, "16-byte tables", nbuf, slot, T);
                expect(L.q_tab == L.m_tab + 16 * (size_t)T, "m_tab holds T int4", nbuf, slot, T);
                expect(L.b_tab == L.q_tab + 16 * (size_t)T, "q_tab holds T float4", nbuf, slot, T);
                expect(L.total == L.b_tab + 2 * wf::kChunk * 4, "b_tab holds 2 kChunk ints",
                       nbuf, slot, T);
                expect(das_lds_fits(L.total, nbuf, slot, T), "exact size fits", nbuf, slot, T);
                expect(!das_lds_fits(L.total - 1, nbuf, slot, T), "one byte short is refused",
                       nbuf, slot, T);
            }
        }
    }
    // A kernel staging two passes per barrier (four window buffers) must
    // refuse the allocation sized for one pass (two buffers): its tables
    // would start where that allocation ends.
    for (int slot : slots)
        for (int T : Ts) {
            const size_t one_pass = das_lds(wf::das_gather_nbuf(1), slot, T).total;
            expect(!das_lds_fits(one_pass, wf::das_gather_nbuf(2), slot, T),
                   "two-pass layout refuses the one-pass size", 4, slot, T);
            expect(das_lds(wf::das_gather_nbuf(2), slot, T).total > one_pass,
                   "two-pass layout is larger", 4, slot, T);
            // the adjoint's window sets are G and H arrays of the same size
            expect(das_lds(wf::das_adjoint_nbuf(2), slot, T).total ==
                       das_lds(wf::das_gather_nbuf(2), slot, T).total,
                   "adjoint sets match gather buffers", 4, slot, T);
        }
    if (failures == 0) std::printf("das_layout: all checks passed\n");
    return failures == 0 ? 0 : 1;
}
