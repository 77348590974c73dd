// saturator.hpp -- e-graph rewriting and code generation of pointwise
// multi-statement programs (include/saturator.h).  Host-only C++.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace stn {
namespace sat {

// Expression node kinds.  FMA(A, B, C) = A + B*C (the paper's notation).
enum Kind : int { K_CONST = 0, K_PARAM, K_LOAD, K_ADD, K_SUB, K_MUL, K_NEG, K_FMA };

inline int arity(int k) {
    switch (k) {
    case K_ADD: case K_SUB: case K_MUL: return 2;
    case K_NEG: return 1;
    case K_FMA: return 3;
    default: return 0;
    }
}

struct Insn {
    int op, a, b, c, d;
};

// A validated program (see include/saturator.h for the instruction set).
struct Program {
    int n_in = 0, n_out = 0, n_par = 0, n_loc = 0, radius = 0;
    std::vector<Insn> insns;
    std::vector<double> consts;
    long long n[3] = {1, 1, 1};
    long long py = 0, pz = 0;  // resolved pitches (never 0 after validation)
};

struct Stats {
    int enodes = 0, eclasses = 0, iterations = 0, saturated = 0;
    double cost_input = 0, cost_extracted = 0;
    int loads = 0, ops = 0, fmas = 0;
    double saturate_ms = 0, extract_ms = 0;
};

struct Generated {
    std::string src, ssa;
    Stats st;
};

enum Form { F_PLAIN = 0, F_CSE = 1, F_CSE_SAT = 2, F_CSE_BULK = 3, F_ACCSAT = 4, F_ACCSAT_Z = 5 };

// Limits of the saturation (the paper's Sec. Experimental Methodology settings).
struct Limits {
    int max_nodes = 10000;
    int max_iters = 10;
    double max_saturate_s = 10.0;
    double max_extract_s = 30.0;
};

// Name of the generated kernel of a form ("sat_kernel_<form>").
const char *kernel_name(int form);

// Check a program; returns "" or the reason it is rejected.
std::string validate(Program &p);

// Rewrite (forms 2, 4, 5), extract and generate HIP source for one form.
// extract: 0 greedy + DAG local search, 1 exhaustive; zb: z planes per
// thread of the streaming form.  Returns "" or an error text; `unsupported`
// is set when the exhaustive extraction is too big.
std::string generate(const Program &p, int form, int extract, int tx, int ty, int zb, const Limits &lim,
                     Generated *out, bool *unsupported);

}  // namespace sat
}  // namespace stn
