// saturator.cpp -- equality saturation of pointwise multi-statement programs.
//
// The steps follow the paper's method (arXiv 2306.13002):
//   * E-graph creation (Sec. "E-Graph Creation"): the postfix program is read
//     into one e-graph in single-assignment form -- every load, parameter,
//     constant and operation becomes an e-node, identical e-nodes share an
//     e-class (hash-consing), local scalars name the e-class of their value.
//   * Rewriting (Sec. "Rewriting Rules", Table tab:rule): FMA1 A+B*C ->
//     FMA(A,B,C), FMA2 A-B*C -> FMA(A,-B,C), FMA3 B*C-A -> FMA(-A,B,C),
//     COMM-ADD, COMM-MUL, ASSOC-ADD1/2, ASSOC-MUL1/2, and constant folding
//     (an e-class analysis: an e-class whose value is a known constant gets
//     a constant e-node).  Matches of one iteration are collected first and
//     applied together, then congruence is restored ("rebuild"); the loop
//     stops when an iteration changes nothing or at the limits of Sec.
//     Experimental Methodology (10 000 e-nodes, 10 iterations, 10 s).
//   * Extraction (Sec. "Code Selection"): the cost model of Sec. "Cost Model"
//     (constant 0, input variable 1, arithmetic 10, memory access 100) is
//     minimized over the selection of one e-node per e-class, counting each
//     e-class once however often it is used (the paper's ILP objective).
//     No ILP solver is used: a bottom-up tree-cost pass gives a first
//     selection and a local search over single e-class switches lowers its
//     DAG cost; an exhaustive search is offered for small e-graphs.
//   * Code generation (Sec. "Code Generation"): one temporary per selected
//     e-node, placed right before its first use, or, in the bulk forms, every
//     load first, in ascending (array, z, y, x) order.
#include "saturator.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <unordered_map>

namespace stn {
namespace sat {
namespace {

using Clock = std::chrono::steady_clock;
double secs_since(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }

uint64_t dbits(double v) {
    uint64_t u;
    std::memcpy(&u, &v, 8);
    return u;
}
double dval(uint64_t u) {
    double v;
    std::memcpy(&v, &u, 8);
    return v;
}

const double kInf = std::numeric_limits<double>::infinity();

enum { OP_CONST = 1, OP_PARAM, OP_LOAD, OP_ADD, OP_SUB, OP_MUL, OP_NEG, OP_STORE, OP_SET, OP_GET };

struct Node {
    int op = K_CONST;
    uint64_t pay = 0;  // CONST: bits of the value; PARAM: index; LOAD: array
    int off[3] = {0, 0, 0};
    int ch[3] = {-1, -1, -1};
    bool operator==(const Node &o) const {
        return op == o.op && pay == o.pay && off[0] == o.off[0] && off[1] == o.off[1] && off[2] == o.off[2] &&
               ch[0] == o.ch[0] && ch[1] == o.ch[1] && ch[2] == o.ch[2];
    }
    bool operator<(const Node &o) const {
        if (op != o.op) return op < o.op;
        if (pay != o.pay) return pay < o.pay;
        for (int i = 0; i < 3; ++i)
            if (off[i] != o.off[i]) return off[i] < o.off[i];
        for (int i = 0; i < 3; ++i)
            if (ch[i] != o.ch[i]) return ch[i] < o.ch[i];
        return false;
    }
};

struct NodeHash {
    size_t operator()(const Node &n) const {
        uint64_t h = 0x9e3779b97f4a7c15ull;
        auto mix = [&h](uint64_t v) { h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2); };
        mix((uint64_t)n.op);
        mix(n.pay);
        for (int i = 0; i < 3; ++i) mix((uint32_t)n.off[i]);
        for (int i = 0; i < 3; ++i) mix((uint32_t)n.ch[i]);
        return (size_t)h;
    }
};

Node mk_const(double v) {
    Node n;
    n.op = K_CONST;
    n.pay = dbits(v);
    return n;
}
Node mk_param(int p) {
    Node n;
    n.op = K_PARAM;
    n.pay = (uint64_t)p;
    return n;
}
Node mk_load(int a, int dx, int dy, int dz) {
    Node n;
    n.op = K_LOAD;
    n.pay = (uint64_t)a;
    n.off[0] = dx;
    n.off[1] = dy;
    n.off[2] = dz;
    return n;
}
Node mk(int op, int a, int b = -1, int c = -1) {
    Node n;
    n.op = op;
    n.ch[0] = a;
    n.ch[1] = b;
    n.ch[2] = c;
    return n;
}

// The paper's cost model: constants 0, input variables 1, memory accesses
// 100, every other operation (here all arithmetic) 10.
double node_cost(int op) {
    switch (op) {
    case K_CONST: return 0;
    case K_PARAM: return 1;
    case K_LOAD: return 100;
    default: return 10;
    }
}

class EGraph {
  public:
    explicit EGraph(bool fold) : fold_(fold) {}

    int find(int x) {
        int r = x;
        while (uf_[r] != r) r = uf_[r];
        while (uf_[x] != r) {
            const int nx = uf_[x];
            uf_[x] = r;
            x = nx;
        }
        return r;
    }

    int add(Node n) {
        n = canon(n);
        auto it = memo_.find(n);
        if (it != memo_.end()) return find(it->second);
        const int id = (int)uf_.size();
        uf_.push_back(id);
        cls_.emplace_back();
        cls_[id].nodes.push_back(n);
        memo_.emplace(n, id);
        ++n_nodes_;
        double v;
        if (fold_ && eval(n, &v)) {
            cls_[id].hc = true;
            cls_[id].cv = v;
            if (n.op != K_CONST) return merge(id, add(mk_const(v)));
        }
        return id;
    }

    int merge(int a, int b) {
        a = find(a);
        b = find(b);
        if (a == b) return a;
        if (cls_[a].nodes.size() < cls_[b].nodes.size()) std::swap(a, b);
        uf_[b] = a;
        Class &A = cls_[a], &B = cls_[b];
        A.nodes.insert(A.nodes.end(), B.nodes.begin(), B.nodes.end());
        std::vector<Node>().swap(B.nodes);
        if (!A.hc && B.hc) {
            A.hc = true;
            A.cv = B.cv;
        }
        return a;
    }

    // Restore the invariants after merges: canonical children, no duplicate
    // e-nodes, congruent e-nodes in one e-class, constants folded.
    void rebuild() {
        bool changed = true;
        while (changed) {
            changed = false;
            memo_.clear();
            for (int c = 0; c < (int)uf_.size(); ++c) {
                if (find(c) != c) continue;
                std::vector<Node> &v = cls_[c].nodes;
                for (Node &n : v) n = canon(n);
                std::sort(v.begin(), v.end());
                v.erase(std::unique(v.begin(), v.end()), v.end());
            }
            for (int c = 0; c < (int)uf_.size(); ++c) {
                if (find(c) != c) continue;
                const std::vector<Node> v = cls_[c].nodes;
                for (const Node &n0 : v) {
                    const Node n = canon(n0);
                    auto it = memo_.find(n);
                    if (it == memo_.end()) {
                        memo_.emplace(n, find(c));
                    } else if (find(it->second) != find(c)) {
                        merge(it->second, c);
                        changed = true;
                    }
                }
            }
            if (changed || !fold_) continue;
            for (int c = 0; c < (int)uf_.size(); ++c) {
                if (find(c) != c) continue;
                if (!cls_[c].hc) {
                    for (const Node &n : cls_[c].nodes) {
                        double v;
                        if (eval(n, &v)) {
                            cls_[c].hc = true;
                            cls_[c].cv = v;
                            break;
                        }
                    }
                }
                if (!cls_[c].hc) continue;
                bool has_node = false;
                for (const Node &n : cls_[c].nodes) has_node |= n.op == K_CONST;
                if (has_node) continue;
                const Node k = mk_const(cls_[c].cv);
                auto it = memo_.find(k);
                if (it != memo_.end()) {
                    merge(it->second, c);
                    changed = true;
                } else {
                    cls_[c].nodes.push_back(k);
                    memo_.emplace(k, c);
                }
            }
        }
        n_nodes_ = 0;
        for (int c = 0; c < (int)uf_.size(); ++c)
            if (find(c) == c) n_nodes_ += cls_[c].nodes.size();
    }

    size_t node_count() const { return n_nodes_; }
    int id_count() const { return (int)uf_.size(); }
    int class_count() {
        int n = 0;
        for (int c = 0; c < (int)uf_.size(); ++c) n += find(c) == c;
        return n;
    }
    const std::vector<Node> &nodes(int c) const { return cls_[c].nodes; }

  private:
    struct Class {
        std::vector<Node> nodes;
        bool hc = false;  // value known to be the constant cv
        double cv = 0;
    };

    Node canon(Node n) {
        for (int i = 0; i < arity(n.op); ++i) n.ch[i] = find(n.ch[i]);
        return n;
    }

    // Constant value of an e-node whose operands are all known constants.
    bool eval(const Node &n, double *v) {
        if (n.op == K_CONST) {
            *v = dval(n.pay);
            return true;
        }
        if (n.op == K_PARAM || n.op == K_LOAD) return false;
        double x[3];
        for (int i = 0; i < arity(n.op); ++i) {
            const Class &c = cls_[find(n.ch[i])];
            if (!c.hc) return false;
            x[i] = c.cv;
        }
        switch (n.op) {
        case K_ADD: *v = x[0] + x[1]; break;
        case K_SUB: *v = x[0] - x[1]; break;
        case K_MUL: *v = x[0] * x[1]; break;
        case K_NEG: *v = -x[0]; break;
        case K_FMA: *v = std::fma(x[1], x[2], x[0]); break;
        default: return false;
        }
        return std::isfinite(*v);
    }

    bool fold_;
    std::vector<int> uf_;
    std::vector<Class> cls_;
    std::unordered_map<Node, int, NodeHash> memo_;
    size_t n_nodes_ = 0;
};

enum Rule { R_COMM_ADD, R_COMM_MUL, R_ASSOC_ADD1, R_ASSOC_ADD2, R_ASSOC_MUL1, R_ASSOC_MUL2, R_FMA1, R_FMA2, R_FMA3 };

struct Match {
    int rule, cls, a, b, c;
};

// One rewrite iteration: collect every match of Table tab:rule, apply them,
// rebuild.  Returns false if the node limit stopped the application.
bool rewrite_once(EGraph &g, const Limits &lim) {
    std::vector<Match> ms;
    for (int c = 0; c < g.id_count(); ++c) {
        if (g.find(c) != c) continue;
        for (const Node &n : g.nodes(c)) {
            const int x = n.ch[0], y = n.ch[1];
            if (n.op == K_ADD) {
                ms.push_back({R_COMM_ADD, c, x, y, -1});
                for (const Node &m : g.nodes(y)) {
                    if (m.op == K_ADD) ms.push_back({R_ASSOC_ADD1, c, x, m.ch[0], m.ch[1]});  // A+(B+C) -> (A+B)+C
                    if (m.op == K_MUL) ms.push_back({R_FMA1, c, x, m.ch[0], m.ch[1]});        // A+B*C -> FMA(A,B,C)
                }
                for (const Node &m : g.nodes(x))
                    if (m.op == K_ADD) ms.push_back({R_ASSOC_ADD2, c, m.ch[0], m.ch[1], y});  // (A+B)+C -> A+(B+C)
            } else if (n.op == K_MUL) {
                ms.push_back({R_COMM_MUL, c, x, y, -1});
                for (const Node &m : g.nodes(y))
                    if (m.op == K_MUL) ms.push_back({R_ASSOC_MUL1, c, x, m.ch[0], m.ch[1]});
                for (const Node &m : g.nodes(x))
                    if (m.op == K_MUL) ms.push_back({R_ASSOC_MUL2, c, m.ch[0], m.ch[1], y});
            } else if (n.op == K_SUB) {
                for (const Node &m : g.nodes(y))
                    if (m.op == K_MUL) ms.push_back({R_FMA2, c, x, m.ch[0], m.ch[1]});  // A-B*C -> FMA(A,-B,C)
                for (const Node &m : g.nodes(x))
                    if (m.op == K_MUL) ms.push_back({R_FMA3, c, y, m.ch[0], m.ch[1]});  // B*C-A -> FMA(-A,B,C)
            }
        }
    }
    for (const Match &m : ms) {
        if (g.node_count() >= (size_t)lim.max_nodes) return false;
        int r = -1;
        switch (m.rule) {
        case R_COMM_ADD: r = g.add(mk(K_ADD, m.b, m.a)); break;
        case R_COMM_MUL: r = g.add(mk(K_MUL, m.b, m.a)); break;
        case R_ASSOC_ADD1: r = g.add(mk(K_ADD, g.add(mk(K_ADD, m.a, m.b)), m.c)); break;
        case R_ASSOC_ADD2: r = g.add(mk(K_ADD, m.a, g.add(mk(K_ADD, m.b, m.c)))); break;
        case R_ASSOC_MUL1: r = g.add(mk(K_MUL, g.add(mk(K_MUL, m.a, m.b)), m.c)); break;
        case R_ASSOC_MUL2: r = g.add(mk(K_MUL, m.a, g.add(mk(K_MUL, m.b, m.c)))); break;
        case R_FMA1: r = g.add(mk(K_FMA, m.a, m.b, m.c)); break;
        case R_FMA2: r = g.add(mk(K_FMA, m.a, g.add(mk(K_NEG, m.b)), m.c)); break;
        case R_FMA3: r = g.add(mk(K_FMA, g.add(mk(K_NEG, m.a)), m.b, m.c)); break;
        }
        g.merge(r, m.cls);
    }
    return true;
}

// ---------------------------------------------------------------------------
// Extraction

struct Selection {
    std::vector<int> sel;  // per e-class id (roots only): index of the chosen e-node, -1 none
};

class DagCost {
  public:
    DagCost(EGraph &g, const std::vector<int> &roots) : g_(g), roots_(roots), seen_(g.id_count(), 0), done_(g.id_count(), 0) {}

    // Cost of the selection, each e-class counted once; kInf if it is cyclic
    // or some reached e-class has no selection.
    double operator()(const std::vector<int> &sel) {
        ++stamp_;
        double total = 0;
        stack_.clear();
        for (int r : roots_) {
            const int c = g_.find(r);
            if (done_[c] == stamp_) continue;
            if (seen_[c] == stamp_) return kInf;
            stack_.push_back({c, 0});
            seen_[c] = stamp_;
            while (!stack_.empty()) {
                Frame &f = stack_.back();
                const int k = sel[f.cls];
                if (k < 0) return kInf;
                const Node &n = g_.nodes(f.cls)[k];
                if (f.next < arity(n.op)) {
                    const int ch = g_.find(n.ch[f.next++]);
                    if (done_[ch] == stamp_) continue;
                    if (seen_[ch] == stamp_) return kInf;  // cycle
                    seen_[ch] = stamp_;
                    stack_.push_back({ch, 0});
                    continue;
                }
                total += node_cost(n.op);
                done_[f.cls] = stamp_;
                stack_.pop_back();
            }
        }
        return total;
    }

    // E-classes reached by the selection (in post-order).
    std::vector<int> reached(const std::vector<int> &sel) {
        std::vector<int> out;
        ++stamp_;
        for (int r : roots_) {
            const int c = g_.find(r);
            if (done_[c] == stamp_) continue;
            stack_.clear();
            stack_.push_back({c, 0});
            seen_[c] = stamp_;
            while (!stack_.empty()) {
                Frame &f = stack_.back();
                const Node &n = g_.nodes(f.cls)[sel[f.cls]];
                if (f.next < arity(n.op)) {
                    const int ch = g_.find(n.ch[f.next++]);
                    if (seen_[ch] == stamp_) continue;
                    seen_[ch] = stamp_;
                    stack_.push_back({ch, 0});
                    continue;
                }
                done_[f.cls] = stamp_;
                out.push_back(f.cls);
                stack_.pop_back();
            }
        }
        return out;
    }

  private:
    struct Frame {
        int cls, next;
    };
    EGraph &g_;
    const std::vector<int> &roots_;
    std::vector<unsigned> seen_, done_;
    unsigned stamp_ = 0;
    std::vector<Frame> stack_;
};

// Bottom-up tree cost: the cheapest e-node of each e-class with every
// e-class priced at its own cheapest tree.
std::vector<int> greedy_selection(EGraph &g) {
    const int N = g.id_count();
    std::vector<double> cost(N, kInf);
    std::vector<int> sel(N, -1);
    bool changed = true;
    while (changed) {
        changed = false;
        for (int c = 0; c < N; ++c) {
            if (g.find(c) != c) continue;
            const std::vector<Node> &v = g.nodes(c);
            for (int k = 0; k < (int)v.size(); ++k) {
                double t = node_cost(v[k].op);
                for (int i = 0; i < arity(v[k].op) && t < kInf; ++i) t += cost[g.find(v[k].ch[i])];
                if (t < cost[c]) {
                    cost[c] = t;
                    sel[c] = k;
                    changed = true;
                }
            }
        }
    }
    return sel;
}

// Lower the DAG cost by local moves: switch one e-class to another e-node,
// or -- since sharing often pays only after two switches (e.g. two FMA2
// rewrites that use the same negated operand) -- switch one e-class so that
// it introduces new e-classes, together with a second reached e-class that
// has an e-node using one of them.  Only moves that lower the cost are kept.
double local_search(EGraph &g, DagCost &dc, std::vector<int> &sel, double max_s, Clock::time_point t0) {
    const int N = g.id_count();
    // users[e] = (d, k): e-node k of e-class d has e-class e as an operand
    std::vector<std::vector<std::pair<int, int>>> users(N);
    for (int d = 0; d < N; ++d) {
        if (g.find(d) != d) continue;
        const std::vector<Node> &v = g.nodes(d);
        for (int k = 0; k < (int)v.size(); ++k)
            for (int i = 0; i < arity(v[k].op); ++i) users[g.find(v[k].ch[i])].push_back({d, k});
    }
    double best = dc(sel);
    std::vector<char> in_reach(N, 0), in_after(N, 0);
    bool improved = true;
    while (improved && secs_since(t0) < max_s) {
        improved = false;
        // one pass over the e-classes reached at its start (a class that is no
        // longer reached after a move is tried harmlessly: its switch changes
        // nothing)
        const std::vector<int> reach = dc.reached(sel);
        std::fill(in_reach.begin(), in_reach.end(), 0);
        for (int x : reach) in_reach[x] = 1;
        for (int c : reach) {
            for (int k = 0; k < (int)g.nodes(c).size(); ++k) {
                if (k == sel[c]) continue;
                const int old = sel[c];
                sel[c] = k;
                const double t = dc(sel);
                if (t < best) {
                    best = t;
                    improved = true;
                    continue;
                }
                // pair moves through the e-classes this switch introduces, tried
                // when the switch alone costs at most one more operation
                bool kept = false;
                if (t <= best + 10) {
                    const std::vector<int> after = dc.reached(sel);
                    for (int x : after) in_after[x] = 1;
                    for (int e : after) {
                        if (in_reach[e] || kept) continue;
                        for (const auto &u : users[e]) {
                            const int d = u.first;
                            if (d == c || !in_after[d] || sel[d] == u.second) continue;
                            const int old_d = sel[d];
                            sel[d] = u.second;
                            const double t2 = dc(sel);
                            if (t2 < best) {
                                best = t2;
                                improved = kept = true;
                                break;
                            }
                            sel[d] = old_d;
                        }
                    }
                    for (int x : after) in_after[x] = 0;
                }
                if (!kept) sel[c] = old;
            }
            if (secs_since(t0) >= max_s) break;
        }
    }
    return best;
}

// Exhaustive minimum over every combination of e-nodes of the e-classes
// that some selection can reach from the roots.
bool exact_selection(EGraph &g, DagCost &dc, const std::vector<int> &roots, std::vector<int> &sel, double *best) {
    const int N = g.id_count();
    std::vector<char> in(N, 0);
    std::vector<int> cl, st;
    for (int r : roots) {
        const int c = g.find(r);
        if (!in[c]) {
            in[c] = 1;
            st.push_back(c);
        }
    }
    while (!st.empty()) {
        const int c = st.back();
        st.pop_back();
        cl.push_back(c);
        for (const Node &n : g.nodes(c))
            for (int i = 0; i < arity(n.op); ++i) {
                const int ch = g.find(n.ch[i]);
                if (!in[ch]) {
                    in[ch] = 1;
                    st.push_back(ch);
                }
            }
    }
    double combos = 1;
    for (int c : cl) combos *= (double)g.nodes(c).size();
    if (combos > (double)(1 << 22)) return false;
    std::vector<int> cur(N, -1);
    for (int c : cl) cur[c] = 0;
    *best = kInf;
    while (true) {
        const double t = dc(cur);
        if (t < *best) {
            *best = t;
            sel = cur;
        }
        size_t i = 0;
        for (; i < cl.size(); ++i) {
            const int c = cl[i];
            if (++cur[c] < (int)g.nodes(c).size()) break;
            cur[c] = 0;
        }
        if (i == cl.size()) break;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Code generation

std::string hexd(double v) {
    char b[64];
    std::snprintf(b, sizeof b, "%a", v);
    return v < 0 ? "(" + std::string(b) + ")" : std::string(b);
}

// A column of the z-streaming form: the loads of one array at one (dx, dy),
// kept in registers w<c>_0 .. w<c>_<dz1-dz0> for z offsets dz0 .. dz1.
struct Column {
    int a, dx, dy, dz0, dz1;
};

struct Emitter {
    const Program &p;
    std::string body, ssa;
    int next = 0;
    int loads = 0, ops = 0, fmas = 0;
    bool stream = false;          // loads read the z-streaming window registers
    std::vector<Column> cols;     // stream: the columns, in load order

    long long offset(int dx, int dy, int dz) const { return (long long)dz * p.pz + (long long)dy * p.py + dx; }
    std::string load_expr(int a, int dx, int dy, int dz) const {
        char b[96];
        if (stream) {
            for (size_t c = 0; c < cols.size(); ++c)
                if (cols[c].a == a && cols[c].dx == dx && cols[c].dy == dy) {
                    std::snprintf(b, sizeof b, "w%zu_%d", c, dz - cols[c].dz0);
                    return b;
                }
        }
        std::snprintf(b, sizeof b, "A.in[%d][o + (%lldLL)]", a, offset(dx, dy, dz));
        return b;
    }
    void line(const std::string &s) { body += "    " + s + "\n"; }
    void ssa_line(const std::string &s) { ssa += s + "\n"; }
};

const char *kOpName[] = {"const", "param", "load", "add", "sub", "mul", "neg", "fma"};

// PLAIN: the statements as written, one expression per statement.
void gen_plain(const Program &p, Emitter &E) {
    struct V {
        std::string expr;
        int ssa;
    };
    std::vector<V> st;
    std::vector<V> loc(p.n_loc);
    std::vector<int> ver(p.n_loc, 0);
    char b[256];
    for (const Insn &in : p.insns) {
        switch (in.op) {
        case OP_CONST: {
            const double v = p.consts[in.a];
            std::snprintf(b, sizeof b, "v%d = const %a", E.next, v);
            E.ssa_line(b);
            st.push_back({hexd(v), E.next++});
            break;
        }
        case OP_PARAM:
            std::snprintf(b, sizeof b, "v%d = param %d", E.next, in.a);
            E.ssa_line(b);
            st.push_back({"A.prm[" + std::to_string(in.a) + "]", E.next++});
            break;
        case OP_LOAD:
            std::snprintf(b, sizeof b, "v%d = load %d %d %d %d", E.next, in.a, in.b, in.c, in.d);
            E.ssa_line(b);
            ++E.loads;
            st.push_back({E.load_expr(in.a, in.b, in.c, in.d), E.next++});
            break;
        case OP_ADD: case OP_SUB: case OP_MUL: {
            const V y = st.back();
            st.pop_back();
            const V x = st.back();
            st.pop_back();
            const char *sym = in.op == OP_ADD ? " + " : (in.op == OP_SUB ? " - " : " * ");
            const char *nm = in.op == OP_ADD ? "add" : (in.op == OP_SUB ? "sub" : "mul");
            std::snprintf(b, sizeof b, "v%d = %s v%d v%d", E.next, nm, x.ssa, y.ssa);
            E.ssa_line(b);
            ++E.ops;
            st.push_back({"(" + x.expr + sym + y.expr + ")", E.next++});
            break;
        }
        case OP_NEG: {
            const V x = st.back();
            st.pop_back();
            std::snprintf(b, sizeof b, "v%d = neg v%d", E.next, x.ssa);
            E.ssa_line(b);
            ++E.ops;
            st.push_back({"(-" + x.expr + ")", E.next++});
            break;
        }
        case OP_GET: st.push_back(loc[in.a]); break;
        case OP_SET: {
            const V x = st.back();
            st.pop_back();
            std::snprintf(b, sizeof b, "l%d_%d", in.a, ver[in.a]++);
            E.line("const double " + std::string(b) + " = " + x.expr + ";");
            loc[in.a] = {b, x.ssa};
            std::snprintf(b, sizeof b, "set %d v%d", in.a, x.ssa);
            E.ssa_line(b);
            break;
        }
        case OP_STORE: {
            const V x = st.back();
            st.pop_back();
            E.line("A.out[" + std::to_string(in.a) + "][o] = " + x.expr + ";");
            std::snprintf(b, sizeof b, "store %d v%d", in.a, x.ssa);
            E.ssa_line(b);
            break;
        }
        }
    }
}

struct Stmt {
    bool store;
    int target, cls;
};

// Read the program into the e-graph.
std::vector<Stmt> load_program(const Program &p, EGraph &g) {
    std::vector<int> st, loc(p.n_loc, -1);
    std::vector<Stmt> out;
    for (const Insn &in : p.insns) {
        switch (in.op) {
        case OP_CONST: st.push_back(g.add(mk_const(p.consts[in.a]))); break;
        case OP_PARAM: st.push_back(g.add(mk_param(in.a))); break;
        case OP_LOAD: st.push_back(g.add(mk_load(in.a, in.b, in.c, in.d))); break;
        case OP_ADD: case OP_SUB: case OP_MUL: {
            const int y = st.back();
            st.pop_back();
            const int x = st.back();
            st.pop_back();
            st.push_back(g.add(mk(in.op == OP_ADD ? K_ADD : (in.op == OP_SUB ? K_SUB : K_MUL), x, y)));
            break;
        }
        case OP_NEG: {
            const int x = st.back();
            st.pop_back();
            st.push_back(g.add(mk(K_NEG, x)));
            break;
        }
        case OP_GET: st.push_back(loc[in.a]); break;
        case OP_SET:
            loc[in.a] = st.back();
            out.push_back({false, in.a, st.back()});
            st.pop_back();
            break;
        case OP_STORE:
            out.push_back({true, in.a, st.back()});
            st.pop_back();
            break;
        }
    }
    return out;
}

// Temporaries for the selected e-nodes, each before its first use; bulk:
// every load first.
void gen_selected(const Program &p, EGraph &g, const std::vector<int> &sel, const std::vector<Stmt> &stmts, bool bulk,
                  Emitter &E) {
    std::vector<int> id(g.id_count(), -1);
    char b[256];
    auto name = [&](int c) { return "_v" + std::to_string(id[g.find(c)]); };
    auto emit_one = [&](int c) {
        const Node &n = g.nodes(c)[sel[c]];
        const int v = E.next++;
        id[c] = v;
        std::string rhs, s;
        switch (n.op) {
        case K_CONST:
            rhs = hexd(dval(n.pay));
            std::snprintf(b, sizeof b, "v%d = const %a", v, dval(n.pay));
            break;
        case K_PARAM:
            rhs = "A.prm[" + std::to_string((int)n.pay) + "]";
            std::snprintf(b, sizeof b, "v%d = param %d", v, (int)n.pay);
            break;
        case K_LOAD:
            rhs = E.load_expr((int)n.pay, n.off[0], n.off[1], n.off[2]);
            std::snprintf(b, sizeof b, "v%d = load %d %d %d %d", v, (int)n.pay, n.off[0], n.off[1], n.off[2]);
            ++E.loads;
            break;
        case K_NEG:
            rhs = "-" + name(n.ch[0]);
            std::snprintf(b, sizeof b, "v%d = neg v%d", v, id[g.find(n.ch[0])]);
            ++E.ops;
            break;
        case K_FMA:
            rhs = "fma(" + name(n.ch[1]) + ", " + name(n.ch[2]) + ", " + name(n.ch[0]) + ")";
            std::snprintf(b, sizeof b, "v%d = fma v%d v%d v%d", v, id[g.find(n.ch[0])], id[g.find(n.ch[1])],
                          id[g.find(n.ch[2])]);
            ++E.ops;
            ++E.fmas;
            break;
        default: {
            const char *sym = n.op == K_ADD ? " + " : (n.op == K_SUB ? " - " : " * ");
            rhs = name(n.ch[0]) + sym + name(n.ch[1]);
            std::snprintf(b, sizeof b, "v%d = %s v%d v%d", v, kOpName[n.op], id[g.find(n.ch[0])], id[g.find(n.ch[1])]);
            ++E.ops;
        }
        }
        E.ssa_line(b);
        E.line("const double _v" + std::to_string(v) + " = " + rhs + ";");
    };
    // iterative post-order emission of the selection below e-class c
    std::vector<std::pair<int, int>> stack;
    auto emit = [&](int c0) {
        c0 = g.find(c0);
        if (id[c0] >= 0) return;
        stack.clear();
        stack.push_back({c0, 0});
        while (!stack.empty()) {
            auto &f = stack.back();
            const Node &n = g.nodes(f.first)[sel[f.first]];
            if (f.second < arity(n.op)) {
                const int ch = g.find(n.ch[f.second++]);
                if (id[ch] < 0) stack.push_back({ch, 0});
                continue;
            }
            if (id[f.first] < 0) emit_one(f.first);
            stack.pop_back();
        }
    };
    if (bulk) {
        std::vector<int> roots;
        for (const Stmt &s : stmts) roots.push_back(s.cls);
        DagCost dc(g, roots);
        std::vector<int> lc;
        for (int c : dc.reached(sel))
            if (g.nodes(c)[sel[c]].op == K_LOAD) lc.push_back(c);
        std::sort(lc.begin(), lc.end(), [&](int a, int c) {
            const Node &x = g.nodes(a)[sel[a]], &y = g.nodes(c)[sel[c]];
            if (x.pay != y.pay) return x.pay < y.pay;
            for (int i = 2; i >= 0; --i)
                if (x.off[i] != y.off[i]) return x.off[i] < y.off[i];
            return false;
        });
        if (E.stream) {  // one window per (array, dx, dy): the z range its loads span
            for (int c : lc) {
                const Node &n = g.nodes(c)[sel[c]];
                bool found = false;
                for (Column &col : E.cols)
                    if (col.a == (int)n.pay && col.dx == n.off[0] && col.dy == n.off[1]) {
                        col.dz0 = std::min(col.dz0, n.off[2]);
                        col.dz1 = std::max(col.dz1, n.off[2]);
                        found = true;
                    }
                if (!found) E.cols.push_back({(int)n.pay, n.off[0], n.off[1], n.off[2], n.off[2]});
            }
        }
        for (int c : lc) emit_one(c);
    }
    for (const Stmt &s : stmts) {
        emit(s.cls);
        if (s.store) {
            E.line("A.out[" + std::to_string(s.target) + "][o] = " + name(s.cls) + ";");
            std::snprintf(b, sizeof b, "store %d v%d", s.target, id[g.find(s.cls)]);
        } else {
            std::snprintf(b, sizeof b, "set %d v%d", s.target, id[g.find(s.cls)]);
        }
        E.ssa_line(b);
    }
}

// Cost of the program as written (every occurrence counted; a local scalar
// read counts as an input variable).
double written_cost(const Program &p) {
    double c = 0;
    for (const Insn &in : p.insns) {
        switch (in.op) {
        case OP_CONST: break;
        case OP_PARAM: case OP_GET: c += 1; break;
        case OP_LOAD: c += 100; break;
        case OP_ADD: case OP_SUB: case OP_MUL: case OP_NEG: c += 10; break;
        default: break;
        }
    }
    return c;
}

const char *kFormName[] = {"PLAIN", "CSE", "CSE+SAT", "CSE+BULK", "ACCSAT", "ACCSAT + z streaming"};

}  // namespace

const char *kernel_name(int form) {
    static const char *names[] = {"sat_kernel_plain", "sat_kernel_cse",    "sat_kernel_cse_sat",
                                  "sat_kernel_cse_bulk", "sat_kernel_accsat", "sat_kernel_accsat_z"};
    return names[form];
}

namespace {

}  // namespace

std::string validate(Program &p) {
    char b[256];
    if (p.n_in < 0 || p.n_in > 128) return "n_inputs must be in [0, 128]";
    if (p.n_out < 1 || p.n_out > 128) return "n_outputs must be in [1, 128]";
    if (p.n_par < 0 || p.n_par > 64) return "n_params must be in [0, 64]";
    if (p.n_loc < 0 || p.n_loc > 256) return "n_locals must be in [0, 256]";
    if (p.radius < 0 || p.radius > 8) return "radius must be in [0, 8]";
    if (p.insns.empty() || p.insns.size() > 65536) return "n_insns must be in [1, 65536]";
    for (double v : p.consts)
        if (!std::isfinite(v)) return "constants must be finite";
    for (int a = 0; a < 3; ++a)
        if (p.n[a] < 1 || p.n[a] > (1LL << 30)) return "interior extents must be in [1, 2^30]";
    const long long PX = p.n[0] + 2 * p.radius, PY = p.n[1] + 2 * p.radius;
    if (p.py == 0) p.py = PX;
    if (p.pz == 0) p.pz = p.py * PY;
    if (p.py < PX) return "pitch_y is smaller than the padded row";
    if (p.pz < p.py * PY) return "pitch_z is smaller than the padded plane";
    std::vector<char> set(p.n_loc, 0);
    int depth = 0, stores = 0;
    for (size_t i = 0; i < p.insns.size(); ++i) {
        const Insn &in = p.insns[i];
        switch (in.op) {
        case OP_CONST:
            if (in.a < 0 || in.a >= (int)p.consts.size()) {
                std::snprintf(b, sizeof b, "insn %zu: constant index %d out of range", i, in.a);
                return b;
            }
            ++depth;
            break;
        case OP_PARAM:
            if (in.a < 0 || in.a >= p.n_par) {
                std::snprintf(b, sizeof b, "insn %zu: parameter index %d out of range", i, in.a);
                return b;
            }
            ++depth;
            break;
        case OP_LOAD:
            if (in.a < 0 || in.a >= p.n_in) {
                std::snprintf(b, sizeof b, "insn %zu: input index %d out of range", i, in.a);
                return b;
            }
            if (std::abs(in.b) > p.radius || std::abs(in.c) > p.radius || std::abs(in.d) > p.radius) {
                std::snprintf(b, sizeof b, "insn %zu: offset (%d,%d,%d) exceeds radius %d", i, in.b, in.c, in.d,
                              p.radius);
                return b;
            }
            ++depth;
            break;
        case OP_ADD: case OP_SUB: case OP_MUL:
            if (depth < 2) {
                std::snprintf(b, sizeof b, "insn %zu: stack underflow", i);
                return b;
            }
            --depth;
            break;
        case OP_NEG:
            if (depth < 1) {
                std::snprintf(b, sizeof b, "insn %zu: stack underflow", i);
                return b;
            }
            break;
        case OP_STORE: case OP_SET:
            if (depth != 1) {
                std::snprintf(b, sizeof b, "insn %zu: a statement must leave exactly one value (has %d)", i, depth);
                return b;
            }
            if (in.op == OP_STORE && (in.a < 0 || in.a >= p.n_out)) {
                std::snprintf(b, sizeof b, "insn %zu: output index %d out of range", i, in.a);
                return b;
            }
            if (in.op == OP_SET) {
                if (in.a < 0 || in.a >= p.n_loc) {
                    std::snprintf(b, sizeof b, "insn %zu: local index %d out of range", i, in.a);
                    return b;
                }
                set[in.a] = 1;
            }
            stores += in.op == OP_STORE;
            depth = 0;
            break;
        case OP_GET:
            if (in.a < 0 || in.a >= p.n_loc || !set[in.a]) {
                std::snprintf(b, sizeof b, "insn %zu: local %d read before it is set", i, in.a);
                return b;
            }
            ++depth;
            break;
        default:
            std::snprintf(b, sizeof b, "insn %zu: unknown op %d", i, in.op);
            return b;
        }
    }
    if (depth != 0) return "the last statement is not terminated by a store or set";
    if (stores == 0) return "the program stores nothing";
    return "";
}

std::string generate(const Program &p, int form, int extract, int tx, int ty, int zb, const Limits &lim,
                     Generated *out, bool *unsupported) {
    *unsupported = false;
    Emitter E{p};
    Stats st;
    st.cost_input = written_cost(p);
    if (form == F_PLAIN) {
        gen_plain(p, E);
        st.cost_extracted = st.cost_input;
    } else {
        const bool rules = form == F_CSE_SAT || form == F_ACCSAT || form == F_ACCSAT_Z;
        const bool bulk = form == F_CSE_BULK || form == F_ACCSAT || form == F_ACCSAT_Z;
        E.stream = form == F_ACCSAT_Z;
        EGraph g(rules);
        std::vector<Stmt> stmts = load_program(p, g);
        const Clock::time_point t0 = Clock::now();
        if (rules) {
            g.rebuild();
            for (int it = 0; it < lim.max_iters; ++it) {
                const size_t n0 = g.node_count();
                const int c0 = g.class_count();
                const bool within = rewrite_once(g, lim);
                g.rebuild();
                st.iterations = it + 1;
                if (g.node_count() == n0 && g.class_count() == c0) {
                    st.saturated = 1;
                    break;
                }
                if (!within || g.node_count() >= (size_t)lim.max_nodes || secs_since(t0) > lim.max_saturate_s) break;
            }
        } else {
            g.rebuild();
            st.saturated = 1;
        }
        st.saturate_ms = 1e3 * secs_since(t0);
        st.enodes = (int)g.node_count();
        st.eclasses = g.class_count();
        std::vector<int> roots;
        for (Stmt &s : stmts) {
            s.cls = g.find(s.cls);
            roots.push_back(s.cls);
        }
        const Clock::time_point t1 = Clock::now();
        DagCost dc(g, roots);
        std::vector<int> sel;
        double cost = 0;
        if (extract == 1) {
            if (!exact_selection(g, dc, roots, sel, &cost)) {
                *unsupported = true;
                return "the e-graph has more than 2^22 selections; exhaustive extraction is not offered";
            }
        } else {
            sel = greedy_selection(g);
            cost = local_search(g, dc, sel, lim.max_extract_s, t1);
        }
        st.extract_ms = 1e3 * secs_since(t1);
        if (!(cost < kInf)) return "extraction found no acyclic selection";
        st.cost_extracted = cost;
        gen_selected(p, g, sel, stmts, bulk, E);
    }
    st.loads = E.loads;
    st.ops = E.ops;
    st.fmas = E.fmas;

    const int NI = std::max(1, p.n_in), NP = std::max(1, p.n_par);
    char b[1024];
    std::string s;
    std::snprintf(b, sizeof b,
                  "// Generated kernel, form %s: e-graph %d e-nodes / %d e-classes after %d iteration(s)%s;\n"
                  "// cost %.0f as written -> %.0f; %d loads, %d operations (%d FMA).\n",
                  kFormName[form], st.enodes, st.eclasses, st.iterations, st.saturated ? " (saturated)" : "",
                  st.cost_input, st.cost_extracted, st.loads, st.ops, st.fmas);
    s += b;
    std::snprintf(b, sizeof b, "struct SatArgs {\n    const double *in[%d];\n    double *out[%d];\n    double prm[%d];\n};\n",
                  NI, p.n_out, NP);
    s += b;
    if (form != F_ACCSAT_Z && zb > 1) {
        // z loop: a thread evaluates planes k0 .. k1-1 of its (i, j) column
        // in turn; every load is issued again, and the planes shared with the
        // previous step come from the caches (same CU, one plane earlier).
        std::snprintf(b, sizeof b,
                      "extern \"C\" __global__ __launch_bounds__(%d) void %s(SatArgs A) {\n"
                      "    const int i = (int)(blockIdx.x * %d + threadIdx.x);\n"
                      "    const int j = (int)(blockIdx.y * %d + threadIdx.y);\n"
                      "    const int k0 = (int)blockIdx.z * %d, k1 = k0 + %d < %lld ? k0 + %d : %lld;\n"
                      "    if (i >= %lld || j >= %lld) return;\n"
                      "    long long o = (long long)(k0 + %d) * %lldLL + (long long)(j + %d) * %lldLL + (i + %d);\n"
                      "#pragma unroll 1\n"
                      "    for (int k = k0; k < k1; ++k, o += %lldLL) {\n",
                      tx * ty, kernel_name(form), tx, ty, zb, zb, p.n[2], zb, p.n[2], p.n[0], p.n[1], p.radius, p.pz,
                      p.radius, p.py, p.radius, p.pz);
        s += b;
        size_t pos = 0;
        while (pos < E.body.size()) {
            const size_t e = E.body.find('\n', pos);
            s += "    " + E.body.substr(pos, e - pos + 1);
            pos = e + 1;
        }
        s += "    }\n}\n";
    } else if (form != F_ACCSAT_Z) {
        std::snprintf(b, sizeof b,
                      "extern \"C\" __global__ __launch_bounds__(%d) void %s(SatArgs A) {\n"
                      "    const int i = (int)(blockIdx.x * %d + threadIdx.x);\n"
                      "    const int j = (int)(blockIdx.y * %d + threadIdx.y);\n"
                      "    const int k = (int)blockIdx.z;\n"
                      "    if (i >= %lld || j >= %lld) return;\n"
                      "    const long long o = (long long)(k + %d) * %lldLL + (long long)(j + %d) * %lldLL + (i + %d);\n",
                      tx * ty, kernel_name(form), tx, ty, p.n[0], p.n[1], p.radius, p.pz, p.radius, p.py, p.radius);
        s += b;
        s += E.body;
        s += "}\n";
    } else {
        // z streaming: a thread walks planes k0 .. k1-1 of its (i, j) column;
        // every load enters a register window at its column's highest z
        // offset and moves down one register per plane until it leaves at
        // the lowest offset.
        std::snprintf(b, sizeof b,
                      "extern \"C\" __global__ __launch_bounds__(%d) void %s(SatArgs A) {\n"
                      "    const int i = (int)(blockIdx.x * %d + threadIdx.x);\n"
                      "    const int j = (int)(blockIdx.y * %d + threadIdx.y);\n"
                      "    const int k0 = (int)blockIdx.z * %d, k1 = k0 + %d < %lld ? k0 + %d : %lld;\n"
                      "    if (i >= %lld || j >= %lld) return;\n"
                      "    long long o = (long long)(k0 + %d) * %lldLL + (long long)(j + %d) * %lldLL + (i + %d);\n",
                      tx * ty, kernel_name(form), tx, ty, zb, zb, p.n[2], zb, p.n[2], p.n[0], p.n[1], p.radius, p.pz,
                      p.radius, p.py, p.radius);
        s += b;
        for (size_t c = 0; c < E.cols.size(); ++c) {
            const Column &col = E.cols[c];
            for (int d = 0; d <= col.dz1 - col.dz0; ++d) {
                std::snprintf(b, sizeof b, "    double w%zu_%d = A.in[%d][o + (%lldLL)];\n", c, d, col.a,
                              E.offset(col.dx, col.dy, col.dz0 + d));
                s += b;
            }
        }
        // The window holds every live value (no separate prefetch registers:
        // with many columns the windows alone fill the register file); the
        // next plane's loads are issued right after the shift, as the last
        // statements of a step, and awaited at their first use.
        s += "    for (int k = k0; k < k1; ++k) {\n";
        size_t pos = 0;
        while (pos < E.body.size()) {
            const size_t e = E.body.find('\n', pos);
            s += "    " + E.body.substr(pos, e - pos + 1);
            pos = e + 1;
        }
        s += "        if (k + 1 < k1) {\n";
        for (size_t c = 0; c < E.cols.size(); ++c) {
            const Column &col = E.cols[c];
            for (int d = 0; d < col.dz1 - col.dz0; ++d) {
                std::snprintf(b, sizeof b, "            w%zu_%d = w%zu_%d;\n", c, d, c, d + 1);
                s += b;
            }
            std::snprintf(b, sizeof b, "            w%zu_%d = A.in[%d][o + (%lldLL)];\n", c, col.dz1 - col.dz0, col.a,
                          E.offset(col.dx, col.dy, col.dz1 + 1));
            s += b;
        }
        std::snprintf(b, sizeof b, "        }\n        o += %lldLL;\n    }\n}\n", p.pz);
        s += b;
    }
    out->src = s;
    out->ssa = E.ssa;
    out->st = st;
    return "";
}

}  // namespace sat
}  // namespace stn
