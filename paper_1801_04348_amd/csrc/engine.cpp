// Symbolic engine: integer polynomials, constraint systems, and the
// comprehensive optimization of Section 3 (Algorithms 1 and 2).
//
// The quintuple Q(S) = (G_C, lambda, omega, gamma, C) follows Section 3.6;
// sequences are stacks with the conventions of Remark 2 (pop takes the head,
// pushing t_1..t_M leaves t_M on top).  A resource counter forks an accept
// branch (0 <= v <= R_i) and a refuse branch (R_i < v) in which the first
// strategy of sigma(r_i) still in omega is applied and r_1..r_i are pushed
// back; a performance counter forks (0 <= v <= P_i) / (P_i < v <= 1) and
// pushes r_1..r_s, p_i.  Inconsistent systems are discarded.
//
// Consistency (Definition 3 (i)) is decided over integers (hypothesis H1):
// the program and data parameters range over the family's finite point set,
// and once they are fixed every constraint of our families is affine in at
// most one machine symbol, so each machine symbol's admissible values form an
// integer interval that is intersected exactly.
#include <algorithm>
#include <cctype>
#include <climits>
#include <sstream>
#include <stdexcept>

#include "pk_internal.hpp"

namespace pk {

// ------------------------------------------------------------------ Poly
Poly Poly::constant(int64_t c) {
    Poly p;
    if (c != 0) p.t[Mono{}] = c;
    return p;
}

Poly Poly::symbol(int id) {
    Poly p;
    p.t[Mono{{id, 1}}] = 1;
    return p;
}

Poly Poly::operator+(const Poly &o) const {
    Poly r = *this;
    for (const auto &kv : o.t) {
        int64_t v = (r.t[kv.first] += kv.second);
        if (v == 0) r.t.erase(kv.first);
    }
    return r;
}

Poly Poly::neg() const {
    Poly r = *this;
    for (auto &kv : r.t) kv.second = -kv.second;
    return r;
}

Poly Poly::operator-(const Poly &o) const { return *this + o.neg(); }

Poly Poly::operator*(const Poly &o) const {
    Poly r;
    for (const auto &a : t)
        for (const auto &b : o.t) {
            std::map<int, int> e;
            for (const auto &f : a.first) e[f.first] += f.second;
            for (const auto &f : b.first) e[f.first] += f.second;
            Mono m(e.begin(), e.end());
            int64_t v = (r.t[m] += a.second * b.second);
            if (v == 0) r.t.erase(m);
        }
    return r;
}

bool Poly::is_const() const {
    for (const auto &kv : t)
        if (!kv.first.empty()) return false;
    return true;
}

int64_t Poly::const_value() const {
    auto it = t.find(Mono{});
    return it == t.end() ? 0 : it->second;
}

int64_t Poly::eval(const std::vector<int64_t> &vals) const {
    int64_t s = 0;
    for (const auto &kv : t) {
        int64_t v = kv.second;
        for (const auto &f : kv.first)
            for (int e = 0; e < f.second; ++e) v *= vals[f.first];
        s += v;
    }
    return s;
}

// ------------------------------------------------------------------ parser
namespace {
struct PolyParser {
    const std::string &s;
    size_t i = 0;
    const std::function<int(const std::string &)> &lookup;
    PolyParser(const std::string &text, const std::function<int(const std::string &)> &lk)
        : s(text), lookup(lk) {}

    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    Poly expr() {
        Poly p = term();
        for (;;) {
            if (eat('+')) p = p + term();
            else if (eat('-')) p = p - term();
            else return p;
        }
    }
    Poly term() {
        Poly p = factor();
        while (eat('*')) p = p * factor();
        return p;
    }
    Poly factor() {
        ws();
        if (eat('-')) return factor().neg();
        Poly p;
        if (eat('(')) {
            p = expr();
            if (!eat(')')) throw std::runtime_error("missing ')' in '" + s + "'");
        } else if (i < s.size() && std::isdigit((unsigned char)s[i])) {
            int64_t v = 0;
            while (i < s.size() && std::isdigit((unsigned char)s[i])) v = v * 10 + (s[i++] - '0');
            p = Poly::constant(v);
        } else if (i < s.size() && (std::isalpha((unsigned char)s[i]) || s[i] == '_')) {
            size_t j = i;
            while (j < s.size() && (std::isalnum((unsigned char)s[j]) || s[j] == '_')) ++j;
            std::string name = s.substr(i, j - i);
            i = j;
            int id = lookup(name);
            if (id < 0) throw std::runtime_error("unknown symbol '" + name + "'");
            p = Poly::symbol(id);
        } else {
            throw std::runtime_error("cannot parse '" + s + "'");
        }
        if (eat('^')) {
            ws();
            int e = 0;
            while (i < s.size() && std::isdigit((unsigned char)s[i])) e = e * 10 + (s[i++] - '0');
            Poly r = Poly::constant(1);
            for (int k = 0; k < e; ++k) r = r * p;
            p = r;
        }
        return p;
    }
};
}  // namespace

Poly parse_poly(const std::string &text, const std::function<int(const std::string &)> &lookup) {
    PolyParser pp(text, lookup);
    Poly p = pp.expr();
    pp.ws();
    if (pp.i != text.size()) throw std::runtime_error("trailing input in '" + text + "'");
    return p;
}

// ------------------------------------------------------------------ family helpers
int Family::sym(const std::string &name) const {
    for (size_t k = 0; k < sym_names.size(); ++k)
        if (sym_names[k] == name) return (int)k;
    return -1;
}

std::string Family::poly_str(const Poly &p) const {
    if (p.t.empty()) return "0";
    std::ostringstream o;
    bool first = true;
    // higher-degree terms first, constants last
    std::vector<std::pair<Mono, int64_t>> terms(p.t.begin(), p.t.end());
    std::stable_sort(terms.begin(), terms.end(),
                     [](const auto &a, const auto &b) { return a.first.size() > b.first.size(); });
    for (const auto &kv : terms) {
        int64_t c = kv.second;
        if (!first) o << (c < 0 ? " - " : " + ");
        else if (c < 0) o << "-";
        int64_t a = c < 0 ? -c : c;
        bool need_star = false;
        if (a != 1 || kv.first.empty()) {
            o << a;
            need_star = true;
        }
        for (const auto &f : kv.first) {
            if (need_star) o << "*";
            o << sym_names[f.first];
            if (f.second != 1) o << "^" << f.second;
            need_star = true;
        }
        first = false;
    }
    return o.str();
}

std::string Family::constraint_str(const Constraint &c) const {
    return poly_str(c.lhs) + (c.strict ? " < " : " <= ") + poly_str(c.rhs);
}

// ------------------------------------------------------------------ consistency
namespace {

// Integer interval with "unbounded" ends.
struct Interval {
    int64_t lo, hi;
    bool empty() const { return lo > hi; }
};

int64_t floor_div(int64_t a, int64_t b) {  // b > 0
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}
int64_t ceil_div(int64_t a, int64_t b) {  // b > 0
    int64_t q = a / b;
    if ((a % b != 0) && (a > 0)) ++q;
    return q;
}

// Substitutes every non-machine symbol, leaving a polynomial in machine
// symbols only.
Poly substitute(const Family &fam, const Poly &p, const std::vector<int64_t> &vals) {
    Poly r;
    for (const auto &kv : p.t) {
        int64_t c = kv.second;
        Mono rest;
        for (const auto &f : kv.first) {
            if (fam.sym_kind[f.first] == SYM_MACHINE) {
                rest.push_back(f);
            } else {
                for (int e = 0; e < f.second; ++e) c *= vals[f.first];
            }
        }
        if (c == 0) continue;
        int64_t v = (r.t[rest] += c);
        if (v == 0) r.t.erase(rest);
    }
    return r;
}

// True when the point (program/data values in `vals`) admits machine values
// satisfying every constraint.  Machine symbols keep their interval domains.
bool point_admits(const Family &fam, const System &C, const std::vector<int64_t> &vals) {
    std::vector<Interval> box(fam.sym_names.size());
    for (size_t k = 0; k < box.size(); ++k) box[k] = Interval{fam.lo[k], fam.hi[k]};
    for (const auto &c : C) {
        Poly d = substitute(fam, c.lhs - c.rhs, vals);  // d <= 0 (or d < 0)
        int64_t bound = c.strict ? -1 : 0;              // integers: d < 0  <=>  d <= -1
        if (d.is_const()) {
            if (d.const_value() > bound) return false;
            continue;
        }
        // affine in a single machine symbol: a*m + b <= bound
        int m = -1;
        int64_t a = 0, b = 0;
        for (const auto &kv : d.t) {
            if (kv.first.empty()) {
                b = kv.second;
            } else if (kv.first.size() == 1 && kv.first[0].second == 1 && (m < 0 || m == kv.first[0].first)) {
                m = kv.first[0].first;
                a += kv.second;
            } else {
                throw std::runtime_error("constraint not affine in one machine symbol: " + fam.constraint_str(c));
            }
        }
        int64_t rhs = bound - b;  // a*m <= rhs
        if (a > 0) box[m].hi = std::min(box[m].hi, floor_div(rhs, a));
        else if (a < 0) box[m].lo = std::max(box[m].lo, ceil_div(-rhs, -a));
        else if (0 > rhs) return false;
        if (box[m].empty()) return false;
    }
    return true;
}

void fill_point(const Family &fam, const std::vector<int64_t> &pt, std::vector<int64_t> *vals) {
    vals->assign(fam.sym_names.size(), 0);
    for (size_t k = 0; k < fam.point_syms.size(); ++k) (*vals)[fam.point_syms[k]] = pt[k];
    for (size_t s = 0; s < fam.sym_names.size(); ++s)
        if (fam.sym_kind[s] == SYM_TABLE) (*vals)[s] = fam.table ? fam.table((int)s, pt) : missing_table_value;
}

}  // namespace

bool consistent(const Family &fam, const System &C) {
    std::vector<int64_t> vals;
    if (fam.points.empty()) {
        fill_point(fam, {}, &vals);
        return point_admits(fam, C, vals);
    }
    for (const auto &pt : fam.points) {
        fill_point(fam, pt, &vals);
        if (point_admits(fam, C, vals)) return true;
    }
    return false;
}

bool system_holds(const Family &fam, const System &C, const std::vector<int64_t> &pt,
                  const std::vector<int64_t> &machine_vals) {
    std::vector<int64_t> vals;
    fill_point(fam, pt, &vals);
    for (size_t s = 0; s < fam.sym_names.size(); ++s)
        if (fam.sym_kind[s] == SYM_MACHINE) vals[s] = machine_vals[s];
    for (const auto &c : C) {
        int64_t l = c.lhs.eval(vals), r = c.rhs.eval(vals);
        if (c.strict ? !(l < r) : !(l <= r)) return false;
    }
    return true;
}

// ------------------------------------------------------------------ Algorithms 1 and 2
namespace {

struct Quintuple {
    std::vector<int> gc;      // source strategies applied (identifies G_C)
    std::vector<int> lam;     // lambda
    std::vector<int> omega;   // unused strategies, O_1 first
    std::deque<int> gamma;    // counters to evaluate, head = next
    System C;
    uint32_t applied = 0;
    std::vector<int> order;
};

using Stack = std::deque<Quintuple>;  // head = front

void push_seq_counters(std::deque<int> *g, const std::vector<int> &items) {
    for (int t : items) g->push_front(t);  // t_1..t_M -> t_M..t_1, s_1..
}

struct Solver {
    const Family &fam;
    std::vector<int> resources;
    explicit Solver(const Family &f) : fam(f) {
        for (size_t c = 0; c < fam.counters.size(); ++c)
            if (!fam.counters[c].performance) resources.push_back((int)c);
    }

    // Algorithm 2
    Stack optimize(Quintuple q) {
        Stack result;
        const int c = q.gamma.front();
        q.gamma.pop_front();
        const CounterDef &cd = fam.counters[c];
        const Poly v = cd.value(q.applied);
        const Poly lim = Poly::symbol(cd.limit);
        Quintuple refuse = q;  // deep copy before the accept constraint is added
        q.C.push_back(Constraint{Poly::constant(0), v, false});
        q.C.push_back(Constraint{v, lim, false});
        result.push_front(std::move(q));
        std::vector<int> pushed;
        if (!cd.performance) {
            refuse.C.push_back(Constraint{lim, v, true});
            for (int r : resources) {
                pushed.push_back(r);
                if (r == c) break;
            }
        } else {
            refuse.C.push_back(Constraint{lim, v, true});
            refuse.C.push_back(Constraint{v, Poly::constant(fam.perf_one), false});
            pushed = resources;
            pushed.push_back(c);
        }
        int chosen = -1;
        for (int o : refuse.omega)
            if (fam.strategies[o].sigma & (1u << c)) {
                chosen = o;
                break;
            }
        if (chosen < 0) return result;
        refuse.omega.erase(std::find(refuse.omega.begin(), refuse.omega.end(), chosen));
        if (fam.strategies[chosen].on_ir) refuse.lam.push_back(chosen);
        else refuse.gc.push_back(chosen);
        refuse.applied |= 1u << chosen;
        refuse.order.push_back(chosen);
        push_seq_counters(&refuse.gamma, pushed);
        Stack sub = optimize(std::move(refuse));
        for (auto &s : sub) result.push_front(std::move(s));  // pushing a sequence
        Stack kept;
        for (auto &s : result)
            if (consistent(fam, s.C)) kept.push_back(std::move(s));
        return kept;
    }

    // Algorithm 1; returns the output stack (head first)
    std::deque<Leaf> run(Quintuple q) {
        std::deque<Leaf> out;
        if (q.gamma.empty()) {
            // processed: ((G_C, lambda), C); inconsistent systems are never output
            if (consistent(fam, q.C)) out.push_back(Leaf{q.applied, q.order, q.lam, q.C});
            return out;
        }
        Stack next = optimize(std::move(q));
        for (auto &qq : next) {
            std::deque<Leaf> sub = run(std::move(qq));
            for (auto &l : sub) out.push_front(std::move(l));
        }
        return out;
    }

    // height of T(Q(S)): one edge per counter evaluation (accept, or refuse
    // when a strategy is available), as in (T1)-(T2)
    int height(Quintuple q) {
        if (q.gamma.empty()) return 0;
        const int c = q.gamma.front();
        q.gamma.pop_front();
        const CounterDef &cd = fam.counters[c];
        Quintuple refuse = q;
        int h = 1 + height(q);
        std::vector<int> pushed;
        if (!cd.performance) {
            for (int r : resources) {
                pushed.push_back(r);
                if (r == c) break;
            }
        } else {
            pushed = resources;
            pushed.push_back(c);
        }
        int chosen = -1;
        for (int o : refuse.omega)
            if (fam.strategies[o].sigma & (1u << c)) {
                chosen = o;
                break;
            }
        if (chosen < 0) return h;
        refuse.omega.erase(std::find(refuse.omega.begin(), refuse.omega.end(), chosen));
        refuse.applied |= 1u << chosen;
        push_seq_counters(&refuse.gamma, pushed);
        return std::max(h, 1 + height(std::move(refuse)));
    }
};

Quintuple initial(const Family &fam) {
    Quintuple q;
    for (size_t o = 0; o < fam.strategies.size(); ++o) q.omega.push_back((int)o);
    for (size_t c = 0; c < fam.counters.size(); ++c) q.gamma.push_back((int)c);
    std::vector<bool> perf(fam.sym_names.size(), false);
    for (const auto &c : fam.counters)
        if (c.performance) perf[c.limit] = true;
    // 0 <= R_i, 0 <= P_i <= 1, 0 <= D_k, 0 <= E_j
    for (int kind : {SYM_MACHINE, SYM_DATA, SYM_PROGRAM})
        for (size_t s = 0; s < fam.sym_names.size(); ++s) {
            if (fam.sym_kind[s] != kind) continue;
            q.C.push_back(Constraint{Poly::constant(0), Poly::symbol((int)s), false});
            if (perf[s]) q.C.push_back(Constraint{Poly::symbol((int)s), Poly::constant(fam.perf_one), false});
        }
    return q;
}

}  // namespace

SolveResult comprehensive_optimization(const Family &fam) {
    Solver s(fam);
    SolveResult r;
    std::deque<Leaf> leaves = s.run(initial(fam));
    r.leaves.assign(leaves.begin(), leaves.end());
    r.height = s.height(initial(fam));
    return r;
}

// ------------------------------------------------------------------ JSON
std::string json_escape(const std::string &s) {
    std::string o;
    for (char c : s) {
        if (c == '"' || c == '\\') {
            o += '\\';
            o += c;
        } else if ((unsigned char)c < 0x20) {
            char buf[8];
            snprintf(buf, sizeof buf, "\\u%04x", c);
            o += buf;
        } else {
            o += c;
        }
    }
    return o;
}

static std::string poly_json(const Family &fam, const Poly &p) {
    std::ostringstream o;
    o << "[";
    bool first = true;
    for (const auto &kv : p.t) {
        if (!first) o << ",";
        first = false;
        o << "[" << kv.second << ",[";
        bool f2 = true;
        for (const auto &f : kv.first) {
            if (!f2) o << ",";
            f2 = false;
            o << "[\"" << json_escape(fam.sym_names[f.first]) << "\"," << f.second << "]";
        }
        o << "]]";
    }
    o << "]";
    return o.str();
}

std::string leaves_json(const Family &fam, const SolveResult &r) {
    std::ostringstream o;
    o << "{\"height\":" << r.height << ",\"leaves\":[";
    for (size_t i = 0; i < r.leaves.size(); ++i) {
        const Leaf &l = r.leaves[i];
        if (i) o << ",";
        o << "{\"variant\":" << l.applied << ",\"applied\":[";
        for (size_t k = 0; k < l.order.size(); ++k)
            o << (k ? "," : "") << "\"" << json_escape(fam.strategies[l.order[k]].name) << "\"";
        o << "],\"lambda\":[";
        for (size_t k = 0; k < l.lam.size(); ++k)
            o << (k ? "," : "") << "\"" << json_escape(fam.strategies[l.lam[k]].name) << "\"";
        o << "],\"system\":[";
        for (size_t k = 0; k < l.C.size(); ++k) {
            const Constraint &c = l.C[k];
            o << (k ? "," : "") << "{\"lhs\":" << poly_json(fam, c.lhs) << ",\"rhs\":" << poly_json(fam, c.rhs)
              << ",\"strict\":" << (c.strict ? "true" : "false") << ",\"text\":\""
              << json_escape(fam.constraint_str(c)) << "\"}";
        }
        o << "]}";
    }
    o << "]}";
    return o.str();
}

// ------------------------------------------------------------------ text families
// One item per line; '#' starts a comment.
Family parse_family(const std::string &spec) {
    Family fam;
    struct ValueLine {
        uint32_t need;
        std::string text;
    };
    std::vector<std::vector<std::pair<uint32_t, Poly>>> values;
    std::vector<std::vector<int64_t>> point_lists;  // per point symbol
    std::vector<std::string> pending_strategy_sigma;
    std::vector<std::vector<std::string>> sigma_names;
    std::vector<std::tuple<std::string, std::vector<std::string>, std::string>> value_lines;

    auto lookup = [&](const std::string &n) { return fam.sym(n); };
    auto add_syms = [&](std::istringstream &ls, int kind) {
        std::string n;
        while (ls >> n) {
            if (fam.sym(n) >= 0) throw std::runtime_error("symbol declared twice: " + n);
            fam.sym_names.push_back(n);
            fam.sym_kind.push_back(kind);
            fam.lo.push_back(0);
            fam.hi.push_back(INT64_MAX / 4);
        }
    };

    std::istringstream in(spec);
    std::string line;
    std::map<int, std::vector<int64_t>> domains;
    while (std::getline(in, line)) {
        auto hash = line.find('#');
        if (hash != std::string::npos) line = line.substr(0, hash);
        std::istringstream ls(line);
        std::string kw;
        if (!(ls >> kw)) continue;
        if (kw == "machine") add_syms(ls, SYM_MACHINE);
        else if (kw == "program") add_syms(ls, SYM_PROGRAM);
        else if (kw == "data") add_syms(ls, SYM_DATA);
        else if (kw == "perf_one") ls >> fam.perf_one;
        else if (kw == "domain" || kw == "points") {
            std::string n;
            ls >> n;
            int id = fam.sym(n);
            if (id < 0) throw std::runtime_error("domain of unknown symbol " + n);
            if (kw == "domain") {
                int64_t lo, hi;
                if (!(ls >> lo >> hi)) throw std::runtime_error("domain needs lo hi: " + line);
                if (fam.sym_kind[id] == SYM_MACHINE) {
                    fam.lo[id] = lo;
                    fam.hi[id] = hi;
                } else {
                    std::vector<int64_t> v;
                    for (int64_t x = lo; x <= hi; ++x) v.push_back(x);
                    domains[id] = v;
                }
            } else {
                std::vector<int64_t> v;
                int64_t x;
                while (ls >> x) v.push_back(x);
                if (fam.sym_kind[id] == SYM_MACHINE) {
                    if (v.empty()) throw std::runtime_error("empty points: " + line);
                    fam.lo[id] = *std::min_element(v.begin(), v.end());
                    fam.hi[id] = *std::max_element(v.begin(), v.end());
                } else {
                    domains[id] = v;
                }
            }
        } else if (kw == "counter") {
            std::string name, kind, lim;
            ls >> name >> kind >> lim;
            CounterDef cd;
            cd.name = name;
            cd.performance = (kind == "performance");
            if (!cd.performance && kind != "resource") throw std::runtime_error("counter kind: " + kind);
            cd.limit = fam.sym(lim);
            if (cd.limit < 0 || fam.sym_kind[cd.limit] != SYM_MACHINE)
                throw std::runtime_error("counter limit must be a machine symbol: " + lim);
            fam.counters.push_back(cd);
            values.emplace_back();
        } else if (kw == "value") {
            std::string name;
            ls >> name;
            std::vector<std::string> need;
            std::string tok;
            while (ls >> tok && tok != ":") need.push_back(tok);
            std::string rest;
            std::getline(ls, rest);
            value_lines.emplace_back(name, need, rest);
        } else if (kw == "strategy") {
            std::string name, where;
            ls >> name >> where;
            StrategyDef sd;
            sd.name = name;
            if (where == "ir") sd.on_ir = true;
            else if (where != "src") throw std::runtime_error("strategy must be src or ir: " + line);
            std::vector<std::string> sig;
            std::string c;
            while (ls >> c) sig.push_back(c);
            fam.strategies.push_back(sd);
            sigma_names.push_back(sig);
        } else {
            throw std::runtime_error("unknown keyword: " + kw);
        }
    }
    if (fam.strategies.size() > 31) throw std::runtime_error("too many strategies");
    auto counter_id = [&](const std::string &n) {
        for (size_t c = 0; c < fam.counters.size(); ++c)
            if (fam.counters[c].name == n) return (int)c;
        throw std::runtime_error("unknown counter " + n);
    };
    auto strategy_id = [&](const std::string &n) {
        for (size_t o = 0; o < fam.strategies.size(); ++o)
            if (fam.strategies[o].name == n) return (int)o;
        throw std::runtime_error("unknown strategy " + n);
    };
    for (size_t o = 0; o < fam.strategies.size(); ++o)
        for (const auto &c : sigma_names[o]) fam.strategies[o].sigma |= 1u << counter_id(c);
    for (const auto &vl : value_lines) {
        int c = counter_id(std::get<0>(vl));
        uint32_t need = 0;
        for (const auto &s : std::get<1>(vl)) need |= 1u << strategy_id(s);
        values[c].emplace_back(need, parse_poly(std::get<2>(vl), lookup));
    }
    for (size_t c = 0; c < fam.counters.size(); ++c) {
        auto entries = values[c];
        std::string name = fam.counters[c].name;
        if (entries.empty()) throw std::runtime_error("counter without value: " + name);
        fam.counters[c].value = [entries, name](uint32_t applied) {
            for (const auto &e : entries)
                if ((e.first & applied) == e.first) return e.second;
            throw std::runtime_error("no value of " + name);
        };
    }
    // the point set: product of the program/data domains
    for (size_t s = 0; s < fam.sym_names.size(); ++s) {
        if (fam.sym_kind[s] == SYM_PROGRAM || fam.sym_kind[s] == SYM_DATA) {
            auto it = domains.find((int)s);
            if (it == domains.end()) throw std::runtime_error("no domain for " + fam.sym_names[s]);
            fam.point_syms.push_back((int)s);
            point_lists.push_back(it->second);
        }
    }
    fam.points.push_back({});
    for (const auto &lst : point_lists) {
        std::vector<std::vector<int64_t>> nxt;
        for (const auto &p : fam.points)
            for (int64_t v : lst) {
                auto q = p;
                q.push_back(v);
                nxt.push_back(q);
            }
        fam.points.swap(nxt);
    }
    return fam;
}

}  // namespace pk
