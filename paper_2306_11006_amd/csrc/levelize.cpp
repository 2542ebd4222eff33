// levelize.cpp -- host-side levelisation of a gate DAG into waves
// (ArctyrEX Section 4.2): Kahn's algorithm with a FIFO of ready gates; a
// gate's wave is one more than the largest wave among the gates producing
// its inputs.  Linear in gates + wires.
#include "../../include/cggi.h"

#include <algorithm>
#include <string>
#include <vector>

namespace cggi {
int set_error(int code, const std::string &msg);
}

namespace {

int n_inputs(int op)
{
    switch (op) {
    case CGGI_NAND: case CGGI_AND: case CGGI_OR: case CGGI_XOR:
    case CGGI_NOR: case CGGI_XNOR:
        return 2;
    case CGGI_MUX:
        return 3;
    case CGGI_NOT: case CGGI_COPY:
        return 1;
    case CGGI_CONST0: case CGGI_CONST1:
        return 0;
    default:
        return -1;
    }
}

} // namespace

extern "C" int cggi_levelize(const cggi_gate_t *gates, int32_t G, int32_t W,
                             int32_t *order, int32_t *level_start,
                             int32_t *n_levels, int32_t *level)
{
    using cggi::set_error;
    if (G < 0 || W < 0)
        return set_error(CGGI_E_SHAPE, "levelize: negative size");
    if ((G > 0 && !gates) || !order || !level_start || !n_levels)
        return set_error(CGGI_E_SHAPE, "levelize: NULL pointer");
    std::vector<int32_t> producer((size_t)W, -1);
    for (int32_t g = 0; g < G; ++g) {
        const cggi_gate_t &gt = gates[g];
        int k = n_inputs(gt.op);
        if (k < 0)
            return set_error(CGGI_E_SHAPE, "levelize: unknown opcode at gate " +
                                               std::to_string(g));
        const int32_t ins[3] = {gt.in0, gt.in1, gt.in2};
        if (gt.out < 0 || gt.out >= W)
            return set_error(CGGI_E_SHAPE, "levelize: output wire out of range "
                                           "at gate " + std::to_string(g));
        for (int i = 0; i < k; ++i) {
            if (ins[i] < 0 || ins[i] >= W)
                return set_error(CGGI_E_SHAPE, "levelize: input wire out of "
                                               "range at gate " +
                                                   std::to_string(g));
            if (ins[i] == gt.out)
                return set_error(CGGI_E_PARAM, "levelize: gate " +
                                                   std::to_string(g) +
                                                   " reads its own output");
        }
        if (producer[gt.out] >= 0)
            return set_error(CGGI_E_PARAM, "levelize: wire " +
                                               std::to_string(gt.out) +
                                               " written twice");
        producer[gt.out] = g;
    }
    // predecessor counts and successor lists (CSR)
    std::vector<int32_t> npred((size_t)G, 0), nsucc((size_t)G + 1, 0);
    for (int32_t g = 0; g < G; ++g) {
        const cggi_gate_t &gt = gates[g];
        const int32_t ins[3] = {gt.in0, gt.in1, gt.in2};
        for (int i = 0; i < n_inputs(gt.op); ++i) {
            int32_t pg = producer[ins[i]];
            if (pg >= 0) {
                ++npred[g];
                ++nsucc[pg + 1];
            }
        }
    }
    for (int32_t g = 0; g < G; ++g)
        nsucc[g + 1] += nsucc[g];
    std::vector<int32_t> succ(nsucc[G]), fill(nsucc.begin(), nsucc.end() - 1);
    for (int32_t g = 0; g < G; ++g) {
        const cggi_gate_t &gt = gates[g];
        const int32_t ins[3] = {gt.in0, gt.in1, gt.in2};
        for (int i = 0; i < n_inputs(gt.op); ++i) {
            int32_t pg = producer[ins[i]];
            if (pg >= 0)
                succ[fill[pg]++] = g;
        }
    }
    // FIFO of ready gates
    std::vector<int32_t> fifo;
    fifo.reserve((size_t)G);
    std::vector<int32_t> lev((size_t)G, 0);
    for (int32_t g = 0; g < G; ++g)
        if (npred[g] == 0)
            fifo.push_back(g);
    for (size_t head = 0; head < fifo.size(); ++head) {
        int32_t g = fifo[head];
        for (int32_t e = nsucc[g]; e < nsucc[g + 1]; ++e) {
            int32_t s = succ[e];
            lev[s] = std::max(lev[s], lev[g] + 1);
            if (--npred[s] == 0)
                fifo.push_back(s);
        }
    }
    if ((int32_t)fifo.size() != G)
        return set_error(CGGI_E_PARAM, "levelize: the gates form a cycle");
    int32_t L = 0;
    for (int32_t g = 0; g < G; ++g)
        L = std::max(L, lev[g] + 1);
    // counting sort by (level, opcode), stable in gate index
    const int NOPS = 11;
    std::vector<int32_t> cnt((size_t)L * NOPS + 1, 0);
    for (int32_t g = 0; g < G; ++g)
        ++cnt[(size_t)lev[g] * NOPS + gates[g].op + 1];
    for (size_t i = 1; i < cnt.size(); ++i)
        cnt[i] += cnt[i - 1];
    for (int32_t l = 0; l <= L; ++l)
        level_start[l] = cnt[(size_t)l * NOPS];
    for (int32_t g = 0; g < G; ++g)
        order[cnt[(size_t)lev[g] * NOPS + gates[g].op]++] = g;
    *n_levels = L;
    if (level)
        for (int32_t g = 0; g < G; ++g)
            level[g] = lev[g];
    return CGGI_OK;
}
