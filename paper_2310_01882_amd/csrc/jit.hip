// Runtime-compiled stencil programs: stencil.apply with an arbitrary
// arithmetic body (Section 2.2 and Listing 2: a region of arith operations
// on constant-offset accesses of input temps; Section 3: the flow discovers
// such regions in Fortran loop nests and extracts them). A small text
// language describes the region; it is parsed here, turned into a z-marching
// HIP kernel and compiled for the device with hipRTC once per program.
//
// Language (grammar and rules are stated in mistencil.h):
//   field u, f;  param c;  profile t;
//   let s = ((((u[1,0,0] + u[-1,0,0]) + u[0,1,0]) + u[0,-1,0]) + u[0,0,1]) + u[0,0,-1];
//   out v = (s - f) * c;
//
// Generated kernels (one module, two entry points): a block owns a
// 64V x 4 (x, y) tile and marches a z-chunk. The vector kernel (V = 2 FP64
// / 4 FP32 cells per lane, whole tiles of fields aligned to V cells) keeps
// one register queue per (field, dy) row over its z offsets and takes x
// neighbours from the adjacent lanes (DPP); the scalar kernel (V = 1, the
// remaining columns or unaligned fields) keeps one queue per (field, dx, dy)
// column. Each queue loads one new level per step, two steps ahead, from a
// level clamped into the halo so the load is unconditional. Every operation
// of the body is emitted fully parenthesised in source order and the
// program is compiled without contraction, so each value is rounded as the
// text says.
#include "ms_internal.hpp"

#include <hip/hiprtc.h>

#include <cctype>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

namespace ms {
namespace {

constexpr int kJitMaxFields = 8, kJitMaxOutputs = 4, kJitMaxParams = 8, kJitMaxProfiles = 4;
constexpr int kJitMaxLets = 256, kJitMaxNodes = 1 << 16, kJitMaxDepth = 200;
constexpr size_t kJitMaxSource = 1 << 16;
constexpr int kJitVecRows = 2;  // rows per lane in the vector kernel

struct Node {
  enum Kind { NUM, FIELD, PARAM, PROFILE, LET, NEG, ADD, SUB, MUL, DIV } kind;
  double num = 0.0;
  int idx = 0;         // field / param / profile / let index
  int dx = 0, dy = 0, dz = 0;
  int a = -1, b = -1;  // operands
};

struct Program {
  std::vector<std::string> fields, params, profiles;
  std::vector<std::string> let_names, out_names;
  std::vector<int> let_root, out_root;
  std::vector<Node> nodes;
};

// ------------------------------------------------------------------ parser

struct ParseError {
  std::string msg;
};

class Parser {
 public:
  explicit Parser(const char* s) : s_(s) {}

  Program run() {
    Program p;
    prog_ = &p;
    skip();
    while (s_[pos_]) {
      const std::string kw = word();
      if (kw == "field" || kw == "param" || kw == "profile") {
        std::vector<std::string>& list =
            kw == "field" ? p.fields : kw == "param" ? p.params : p.profiles;
        do {
          const std::string n = name();
          declare(n);
          list.push_back(n);
        } while (accept(','));
        const size_t cap = kw == "field" ? kJitMaxFields
                           : kw == "param" ? kJitMaxParams
                                           : kJitMaxProfiles;
        if (list.size() > cap) fail("too many " + kw + " declarations");
      } else if (kw == "let" || kw == "out") {
        const std::string n = name();
        expect('=');
        depth_ = 0;
        const int root = expr();
        declare(n);
        if (kw == "let") {
          p.let_names.push_back(n);
          p.let_root.push_back(root);
          if (p.let_names.size() > (size_t)kJitMaxLets) fail("too many let statements");
        } else {
          p.out_names.push_back(n);
          p.out_root.push_back(root);
          if (p.out_names.size() > (size_t)kJitMaxOutputs) fail("too many outputs");
        }
      } else {
        fail(kw.empty() ? "expected a statement" : "unknown statement '" + kw + "'");
      }
      expect(';');
    }
    if (p.out_names.empty()) fail("the program has no output");
    return p;
  }

 private:
  const char* s_;
  size_t pos_ = 0;
  int depth_ = 0;
  Program* prog_ = nullptr;
  std::set<std::string> names_;

  [[noreturn]] void fail(const std::string& m) {
    int line = 1, col = 1;
    for (size_t i = 0; i < pos_ && s_[i]; ++i) {
      if (s_[i] == '\n') {
        ++line;
        col = 1;
      } else {
        ++col;
      }
    }
    throw ParseError{"line " + std::to_string(line) + " col " + std::to_string(col) + ": " + m};
  }

  void skip() {
    for (;;) {
      while (s_[pos_] && std::isspace((unsigned char)s_[pos_])) ++pos_;
      if (s_[pos_] != '#') return;
      while (s_[pos_] && s_[pos_] != '\n') ++pos_;
    }
  }
  bool accept(char c) {
    if (s_[pos_] != c) return false;
    ++pos_;
    skip();
    return true;
  }
  void expect(char c) {
    if (!accept(c)) fail(std::string("expected '") + c + "'");
  }
  std::string word() {
    std::string w;
    if (std::isalpha((unsigned char)s_[pos_]) || s_[pos_] == '_')
      while (std::isalnum((unsigned char)s_[pos_]) || s_[pos_] == '_') w += s_[pos_++];
    skip();
    return w;
  }
  std::string name() {
    const std::string n = word();
    if (n.empty()) fail("expected a name");
    return n;
  }
  void declare(const std::string& n) {
    static const char* kReserved[] = {"field", "param", "profile", "let", "out"};
    for (const char* r : kReserved)
      if (n == r) fail("'" + n + "' is a reserved word");
    if (!names_.insert(n).second) fail("'" + n + "' is already defined");
  }
  int add(const Node& n) {
    if (prog_->nodes.size() >= (size_t)kJitMaxNodes) fail("program too large");
    prog_->nodes.push_back(n);
    return (int)prog_->nodes.size() - 1;
  }
  int binary(Node::Kind k, int a, int b) {
    Node n;
    n.kind = k;
    n.a = a;
    n.b = b;
    return add(n);
  }
  int find(const std::vector<std::string>& v, const std::string& n) {
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i] == n) return (int)i;
    return -1;
  }
  int offset() {
    const bool neg = accept('-');
    if (!std::isdigit((unsigned char)s_[pos_])) fail("expected an integer offset");
    int v = 0;
    while (std::isdigit((unsigned char)s_[pos_])) {
      v = v * 10 + (s_[pos_++] - '0');
      if (v > 1000) fail("offset out of range");
    }
    skip();
    v = neg ? -v : v;
    if (v < -1 || v > 1) fail("offsets must lie in [-1, 1] (halo width 1)");
    return v;
  }

  int expr() {
    if (++depth_ > kJitMaxDepth) fail("expression nested too deeply");
    int l = term();
    for (;;) {
      if (accept('+')) l = binary(Node::ADD, l, term());
      else if (accept('-')) l = binary(Node::SUB, l, term());
      else break;
    }
    --depth_;
    return l;
  }
  int term() {
    int l = unary();
    for (;;) {
      if (accept('*')) l = binary(Node::MUL, l, unary());
      else if (accept('/')) l = binary(Node::DIV, l, unary());
      else break;
    }
    return l;
  }
  int unary() {
    if (accept('-')) {
      if (++depth_ > kJitMaxDepth) fail("expression nested too deeply");
      const int a = unary();
      --depth_;
      return binary(Node::NEG, a, -1);
    }
    return primary();
  }
  int primary() {
    if (accept('(')) {
      const int e = expr();
      expect(')');
      return e;
    }
    const char c = s_[pos_];
    if (std::isdigit((unsigned char)c) || c == '.') {
      const char* start = s_ + pos_;
      // decimal literal: digits [. digits] [e|E [+|-] digits]
      size_t p = pos_;
      bool digits = false;
      while (std::isdigit((unsigned char)s_[p])) ++p, digits = true;
      if (s_[p] == '.') {
        ++p;
        while (std::isdigit((unsigned char)s_[p])) ++p, digits = true;
      }
      if (!digits) fail("malformed number");
      if (s_[p] == 'e' || s_[p] == 'E') {
        size_t q = p + 1;
        if (s_[q] == '+' || s_[q] == '-') ++q;
        if (!std::isdigit((unsigned char)s_[q])) fail("malformed exponent");
        while (std::isdigit((unsigned char)s_[q])) ++q;
        p = q;
      }
      if (std::isalpha((unsigned char)s_[p]) || s_[p] == '_') fail("malformed number");
      const std::string text(start, s_ + p);
      const double v = std::strtod(text.c_str(), nullptr);
      if (!std::isfinite(v)) fail("constant out of range");
      pos_ = p;
      skip();
      Node n;
      n.kind = Node::NUM;
      n.num = v;
      return add(n);
    }
    const std::string id = word();
    if (id.empty()) fail("expected a number, a name or '('");
    Node n;
    int k;
    if ((k = find(prog_->fields, id)) >= 0) {
      n.kind = Node::FIELD;
      n.idx = k;
      if (accept('[')) {
        n.dx = offset();
        expect(',');
        n.dy = offset();
        expect(',');
        n.dz = offset();
        expect(']');
      }
    } else if ((k = find(prog_->params, id)) >= 0) {
      n.kind = Node::PARAM;
      n.idx = k;
    } else if ((k = find(prog_->profiles, id)) >= 0) {
      n.kind = Node::PROFILE;
      n.idx = k;
    } else if ((k = find(prog_->let_names, id)) >= 0) {
      n.kind = Node::LET;
      n.idx = k;
    } else {
      fail("'" + id + "' is not defined (outputs cannot be read)");
    }
    if (n.kind != Node::FIELD && s_[pos_] == '[') fail("only fields take offsets");
    return add(n);
  }
};

// ----------------------------------------------------------------- codegen

struct Column {
  int field, dx, dy;
  int dmin, dmax;  // z offsets read
};

std::string hex_literal(double v, int dtype) {
  char buf[64];
  if (dtype == MS_F64) {
    std::snprintf(buf, sizeof buf, "%a", v);
  } else {
    const float f = (float)v;  // round to nearest, like a conversion at run time
    std::snprintf(buf, sizeof buf, "%af", (double)f);
  }
  return buf;
}

struct Codegen {
  const Program& p;
  int dtype;
  std::vector<Column> cols;
  std::map<std::pair<int, std::pair<int, int>>, int> col_of;

  int column(int f, int dx, int dy) {
    auto key = std::make_pair(f, std::make_pair(dx, dy));
    auto it = col_of.find(key);
    if (it != col_of.end()) return it->second;
    cols.push_back({f, dx, dy, 2, -2});
    col_of[key] = (int)cols.size() - 1;
    return (int)cols.size() - 1;
  }

  static std::string qname(int c, int d) {
    return "q" + std::to_string(c) + (d < 0 ? "m" : "p") + std::to_string(d < 0 ? -d : d);
  }

  std::string emit(int id) {
    const Node& n = p.nodes[id];
    switch (n.kind) {
      case Node::NUM: return "((T)" + hex_literal(n.num, dtype) + ")";
      case Node::FIELD: {
        const int c = col_of.at(std::make_pair(n.idx, std::make_pair(n.dx, n.dy)));
        return qname(c, n.dz);
      }
      case Node::PARAM: return "prm" + std::to_string(n.idx);
      case Node::PROFILE: return "pf" + std::to_string(n.idx);
      case Node::LET: return "t" + std::to_string(n.idx);
      case Node::NEG: return "(-" + emit(n.a) + ")";
      case Node::ADD: return "(" + emit(n.a) + " + " + emit(n.b) + ")";
      case Node::SUB: return "(" + emit(n.a) + " - " + emit(n.b) + ")";
      case Node::MUL: return "(" + emit(n.a) + " * " + emit(n.b) + ")";
      case Node::DIV: return "(" + emit(n.a) + " / " + emit(n.b) + ")";
    }
    return "";
  }

  std::set<int> prof_used;

  // The scalar kernel: one x cell per lane, columns x0 .. nx-1.
  std::string run() {
    std::set<int> prm_used;
    for (const Node& n : p.nodes) {
      if (n.kind == Node::FIELD) {
        Column& c = cols[column(n.idx, n.dx, n.dy)];
        c.dmin = std::min(c.dmin, n.dz);
        c.dmax = std::max(c.dmax, n.dz);
      } else if (n.kind == Node::PARAM) {
        prm_used.insert(n.idx);
      } else if (n.kind == Node::PROFILE) {
        prof_used.insert(n.idx);
      }
    }
    std::string o;
    o += "extern \"C\" __global__ __launch_bounds__(256) void ms_jit_kernel_s(JitArgs a) {\n"
         "  const int b = blockIdx.x, nb = a.nblocks;\n"
         "  const int xcd = b & 7, slot = b >> 3, qn = nb >> 3, rn = nb & 7;\n"
         "  const int tile = xcd * qn + (xcd < rn ? xcd : rn) + slot;\n"
         "  const int txi = tile % a.tiles_x, rest = tile / a.tiles_x;\n"
         "  const int tyi = rest % a.tiles_y, tzi = rest / a.tiles_y;\n"
         "  const int i = a.x0 + txi * 64 + (int)(threadIdx.x & 63);\n"
         "  const int j = tyi * 4 + (int)(threadIdx.x >> 6);\n"
         "  if (i >= a.nx || j >= a.ny) return;\n"
         "  const int nz = a.nz, z0 = tzi * a.zc;\n"
         "  const int z1 = z0 + a.zc < nz ? z0 + a.zc : nz;\n"
         "  const long long sy = a.sy, sz = a.sz;\n"
         "  const long long base = (long long)(j + 1) * sy + (i + 1);\n"
         "  auto lev = [&](int l) { return (long long)((l < nz ? l : nz) + 1) * sz; };\n";
    for (int k : prm_used) o += "  const T prm" + std::to_string(k) + " = a.prm[" + std::to_string(k) + "];\n";
    for (size_t c = 0; c < cols.size(); ++c) {
      const Column& q = cols[c];
      const std::string cs = std::to_string(c);
      o += "  const T* __restrict__ c" + cs + " = a.in[" + std::to_string(q.field) + "] + base + (" +
           std::to_string(q.dy) + ") * sy + (" + std::to_string(q.dx) + ");\n";
      for (int d = q.dmin; d <= q.dmax; ++d)
        o += "  T " + qname((int)c, d) + " = c" + cs + "[lev(z0 + (" + std::to_string(d) + "))];\n";
      o += "  T n" + cs + "a = c" + cs + "[lev(z0 + " + std::to_string(q.dmax + 1) + ")];\n";
      o += "  T n" + cs + "b = c" + cs + "[lev(z0 + " + std::to_string(q.dmax + 2) + ")];\n";
    }
    // Two steps per trip, so the two prefetch registers of a column swap
    // roles instead of being copied: a copy of a register whose load is
    // still in flight would wait for that load.
    o += "  for (int k = z0; k < z1; k += 2) {\n";
    o += step("k", 'a', "    ");
    o += "    if (k + 1 >= z1) break;\n";
    o += "    {\n      const int k1 = k + 1;\n";
    o += step("k1", 'b', "      ");
    o += "    }\n";
    o += "  }\n}\n";
    return o;
  }

  // One z step at level `k`: profiles, lets, outputs and their stores, then
  // the queue rotation; prefetch register `ph` takes the level two steps on.
  std::string step(const std::string& k, char ph, const std::string& in) {
    std::string o;
    for (int q = 0; q < (int)p.profiles.size(); ++q)
      if (prof_used.count(q))
        o += in + "const T pf" + std::to_string(q) + " = a.prof[" + std::to_string(q) + "][" + k + "];\n";
    for (size_t l = 0; l < p.let_root.size(); ++l)
      o += in + "const T t" + std::to_string(l) + " = " + emit(p.let_root[l]) + ";\n";
    for (size_t r = 0; r < p.out_root.size(); ++r) {
      const std::string rs = std::to_string(r);
      o += in + "const T o" + rs + " = " + emit(p.out_root[r]) + ";\n";
      o += in + "__builtin_nontemporal_store(o" + rs + ", a.out[" + rs + "] + (long long)(" + k +
           " + 1) * sz + base);\n";
    }
    for (size_t c = 0; c < cols.size(); ++c) {
      const Column& q = cols[c];
      const std::string cs = std::to_string(c), reg = "n" + cs + ph;
      for (int d = q.dmin; d < q.dmax; ++d)
        o += in + "" + qname((int)c, d) + " = " + qname((int)c, d + 1) + ";\n";
      o += in + "" + qname((int)c, q.dmax) + " = " + reg + ";\n";
      o += in + "" + reg + " = c" + cs + "[lev(" + k + " + " + std::to_string(q.dmax + 3) + ")];\n";
    }
    return o;
  }
};

// The vector kernel: V consecutive x cells of R rows per lane (one 16-byte
// load per row and level), whole 64V-column tiles only. A row the body
// reads at several y offsets is loaded once for the lane's R rows. Accesses
// with dx = -1 / +1 take the neighbour lane's last / first element through
// a DPP move; lanes 0 and 63 take the cell beyond the wave from one extra
// load per row and level (every other lane loads its own first cell there,
// a cache hit).
struct VecCodegen {
  const Program& p;
  int dtype, V, R;
  struct Group {
    int field, row, dmin, dmax;  // row: offset from the lane's first row
    bool edge;
  };
  std::vector<Group> groups;
  std::map<std::pair<int, int>, int> group_of;
  std::set<int> prm_used, prof_used;
  std::set<std::pair<int, int>> lused, rused;  // (group, dz) read at dx -1 / +1

  static std::string gname(int g, int d) {
    return "g" + std::to_string(g) + (d < 0 ? "m" : "p") + std::to_string(d < 0 ? -d : d);
  }
  static std::string ename(int g, int d) { return "e" + gname(g, d).substr(1); }

  std::string emit(int id, int v, int r) {
    const Node& n = p.nodes[id];
    switch (n.kind) {
      case Node::NUM: return "((T)" + hex_literal(n.num, dtype) + ")";
      case Node::FIELD: {
        const int g = group_of.at(std::make_pair(n.idx, r + n.dy));
        const std::string q = gname(g, n.dz);
        if (n.dx == 0) return q + "[" + std::to_string(v) + "]";
        if (n.dx < 0) return v > 0 ? q + "[" + std::to_string(v - 1) + "]" : "L" + q.substr(1);
        return v < V - 1 ? q + "[" + std::to_string(v + 1) + "]" : "R" + q.substr(1);
      }
      case Node::PARAM: return "prm" + std::to_string(n.idx);
      case Node::PROFILE: return "pf" + std::to_string(n.idx);
      case Node::LET:
        return "t" + std::to_string(n.idx) + "_" + std::to_string(r) + "_" + std::to_string(v);
      case Node::NEG: return "(-" + emit(n.a, v, r) + ")";
      case Node::ADD: return "(" + emit(n.a, v, r) + " + " + emit(n.b, v, r) + ")";
      case Node::SUB: return "(" + emit(n.a, v, r) + " - " + emit(n.b, v, r) + ")";
      case Node::MUL: return "(" + emit(n.a, v, r) + " * " + emit(n.b, v, r) + ")";
      case Node::DIV: return "(" + emit(n.a, v, r) + " / " + emit(n.b, v, r) + ")";
    }
    return "";
  }

  std::string step(const std::string& k, char ph, const std::string& in) {
    std::string o;
    for (int q : prof_used)
      o += in + "const T pf" + std::to_string(q) + " = a.prof[" + std::to_string(q) + "][" + k + "];\n";
    for (auto gd : lused)
      o += in + "const T L" + gname(gd.first, gd.second).substr(1) + " = ms_from_left(" +
           ename(gd.first, gd.second) + ", " + gname(gd.first, gd.second) + "[" +
           std::to_string(V - 1) + "]);\n";
    for (auto gd : rused)
      o += in + "const T R" + gname(gd.first, gd.second).substr(1) + " = ms_from_right(" +
           ename(gd.first, gd.second) + ", " + gname(gd.first, gd.second) + "[0]);\n";
    for (int r = 0; r < R; ++r) {
      for (size_t l = 0; l < p.let_root.size(); ++l)
        for (int v = 0; v < V; ++v)
          o += in + "const T t" + std::to_string(l) + "_" + std::to_string(r) + "_" +
               std::to_string(v) + " = " + emit(p.let_root[l], v, r) + ";\n";
      o += in + "if (j + " + std::to_string(r) + " < a.ny) {\n";
      for (size_t q = 0; q < p.out_root.size(); ++q) {
        o += in + "  {\n" + in + "    TV ov;\n";
        for (int v = 0; v < V; ++v)
          o += in + "    ov[" + std::to_string(v) + "] = " + emit(p.out_root[q], v, r) + ";\n";
        o += in + "    __builtin_nontemporal_store(ov, (TV*)(a.out[" + std::to_string(q) +
             "] + (long long)(" + k + " + 1) * sz + base + " + std::to_string(r) + " * sy));\n" +
             in + "  }\n";
      }
      o += in + "}\n";
    }
    for (size_t g = 0; g < groups.size(); ++g) {
      const Group& q = groups[g];
      const std::string gs = std::to_string(g), reg = std::string(1, ph);
      for (int d = q.dmin; d < q.dmax; ++d) {
        o += in + gname((int)g, d) + " = " + gname((int)g, d + 1) + ";\n";
        if (q.edge) o += in + ename((int)g, d) + " = " + ename((int)g, d + 1) + ";\n";
      }
      o += in + gname((int)g, q.dmax) + " = n" + gs + reg + ";\n";
      o += in + "n" + gs + reg + " = *(const TV*)(c" + gs + " + lev(" + k + " + " +
           std::to_string(q.dmax + 3) + "));\n";
      if (q.edge) {
        o += in + ename((int)g, q.dmax) + " = m" + gs + reg + ";\n";
        o += in + "m" + gs + reg + " = c" + gs + "[lev(" + k + " + " + std::to_string(q.dmax + 3) +
             ") + eoff];\n";
      }
    }
    return o;
  }

  std::string run() {
    for (const Node& n : p.nodes) {
      if (n.kind == Node::FIELD) {
        for (int r = 0; r < R; ++r) {
          auto key = std::make_pair(n.idx, r + n.dy);
          if (!group_of.count(key)) {
            group_of[key] = (int)groups.size();
            groups.push_back({n.idx, r + n.dy, 2, -2, false});
          }
          const int gi = group_of[key];
          Group& g = groups[gi];
          g.dmin = std::min(g.dmin, n.dz);
          g.dmax = std::max(g.dmax, n.dz);
          if (n.dx != 0) {
            g.edge = true;
            (n.dx < 0 ? lused : rused).insert(std::make_pair(gi, n.dz));
          }
        }
      } else if (n.kind == Node::PARAM) {
        prm_used.insert(n.idx);
      } else if (n.kind == Node::PROFILE) {
        prof_used.insert(n.idx);
      }
    }
    const std::string Vs = std::to_string(V), Rs = std::to_string(R);
    std::string o = "typedef T TV __attribute__((ext_vector_type(" + Vs + ")));\n";
    o += "extern \"C\" __global__ __launch_bounds__(256) void ms_jit_kernel_v(JitArgs a) {\n"
         "  const int b = blockIdx.x, nb = a.nblocks;\n"
         "  const int xcd = b & 7, slot = b >> 3, qn = nb >> 3, rn = nb & 7;\n"
         "  const int tile = xcd * qn + (xcd < rn ? xcd : rn) + slot;\n"
         "  const int txi = tile % a.tiles_x, rest = tile / a.tiles_x;\n"
         "  const int tyi = rest % a.tiles_y, tzi = rest / a.tiles_y;\n"
         "  const int lane = (int)(threadIdx.x & 63);\n"
         "  const int i = txi * " + std::to_string(64 * V) + " + " + Vs + " * lane;\n"
         "  const int j = tyi * " + std::to_string(4 * R) + " + " + Rs + " * (int)(threadIdx.x >> 6);\n"
         "  if (j >= a.ny) return;  // whole waves only: the DPP moves stay within a wave\n"
         "  const int eoff = lane == 0 ? -1 : (lane == 63 ? " + Vs + " : 0);\n"
         "  const int nz = a.nz, ny = a.ny, z0 = tzi * a.zc;\n"
         "  const int z1 = z0 + a.zc < nz ? z0 + a.zc : nz;\n"
         "  const long long sy = a.sy, sz = a.sz;\n"
         "  const long long base = (long long)(j + 1) * sy + (i + 1);\n"
         "  auto lev = [&](int l) { return (long long)((l < nz ? l : nz) + 1) * sz; };\n"
         "  // a row's offset from row j, clamped into the halo (rows past ny\n"
         "  // feed no stored cell)\n"
         "  auto rowoff = [&](int d) { return (long long)((j + d < ny ? j + d : ny) - j) * sy; };\n";
    for (int k : prm_used) o += "  const T prm" + std::to_string(k) + " = a.prm[" + std::to_string(k) + "];\n";
    for (size_t g = 0; g < groups.size(); ++g) {
      const Group& q = groups[g];
      const std::string gs = std::to_string(g);
      o += "  const T* __restrict__ c" + gs + " = a.in[" + std::to_string(q.field) +
           "] + base + rowoff(" + std::to_string(q.row) + ");\n";
      for (int d = q.dmin; d <= q.dmax; ++d) {
        o += "  TV " + gname((int)g, d) + " = *(const TV*)(c" + gs + " + lev(z0 + (" +
             std::to_string(d) + ")));\n";
        if (q.edge)
          o += "  T " + ename((int)g, d) + " = c" + gs + "[lev(z0 + (" + std::to_string(d) +
               ")) + eoff];\n";
      }
      for (int t = 0; t < 2; ++t) {
        const std::string reg = t ? "b" : "a", lv = std::to_string(q.dmax + 1 + t);
        o += "  TV n" + gs + reg + " = *(const TV*)(c" + gs + " + lev(z0 + " + lv + "));\n";
        if (q.edge) o += "  T m" + gs + reg + " = c" + gs + "[lev(z0 + " + lv + ") + eoff];\n";
      }
    }
    o += "  for (int k = z0; k < z1; k += 2) {\n";
    o += step("k", 'a', "    ");
    o += "    if (k + 1 >= z1) break;\n";
    o += "    {\n      const int k1 = k + 1;\n";
    o += step("k1", 'b', "      ");
    o += "    }\n  }\n}\n";
    return o;
  }
};

// The generated source: shared declarations, the scalar kernel and the
// vector kernel (2 FP64 / 4 FP32 cells per lane).
std::string generate(const Program& p, int dtype) {
  std::string o = dtype == MS_F64 ? "typedef double T;\n" : "typedef float T;\n";
  o += "struct JitArgs {\n"
       "  const T* in[8];\n  T* out[4];\n  const T* prof[4];\n  T prm[8];\n"
       "  long long sy, sz;\n  int nx, ny, nz, zc;\n  int tiles_x, tiles_y, nblocks, x0;\n"
       "};\n";
  // lane l receives lane l-1's value (lane 0 keeps `old`), or lane l+1's
  // (lane 63 keeps `old`): DPP wave_shr:1 / wave_shl:1 on each 32-bit half
  const char* dpp = dtype == MS_F64 ?
      "__device__ __forceinline__ T ms_dpp(T old, T v, int ctl_shr) {\n"
      "  const long long o = __builtin_bit_cast(long long, old), s = __builtin_bit_cast(long long, v);\n"
      "  int lo, hi;\n"
      "  if (ctl_shr) {\n"
      "    lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x138, 0xf, 0xf, false);\n"
      "    hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x138, 0xf, 0xf, false);\n"
      "  } else {\n"
      "    lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x130, 0xf, 0xf, false);\n"
      "    hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x130, 0xf, 0xf, false);\n"
      "  }\n"
      "  return __builtin_bit_cast(T, ((long long)hi << 32) | (unsigned int)lo);\n"
      "}\n" :
      "__device__ __forceinline__ T ms_dpp(T old, T v, int ctl_shr) {\n"
      "  const int o = __builtin_bit_cast(int, old), s = __builtin_bit_cast(int, v);\n"
      "  const int r = ctl_shr ? __builtin_amdgcn_update_dpp(o, s, 0x138, 0xf, 0xf, false)\n"
      "                        : __builtin_amdgcn_update_dpp(o, s, 0x130, 0xf, 0xf, false);\n"
      "  return __builtin_bit_cast(T, r);\n"
      "}\n";
  o += dpp;
  o += "__device__ __forceinline__ T ms_from_left(T old, T v) { return ms_dpp(old, v, 1); }\n"
       "__device__ __forceinline__ T ms_from_right(T old, T v) { return ms_dpp(old, v, 0); }\n";
  o += Codegen{p, dtype}.run();
  o += VecCodegen{p, dtype, dtype == MS_F64 ? 2 : 4, kJitVecRows}.run();
  return o;
}

// Host mirror of the generated JitArgs (same member order and types).
template <typename T>
struct JitArgs {
  const T* in[kJitMaxFields];
  T* out[kJitMaxOutputs];
  const T* prof[kJitMaxProfiles];
  T prm[kJitMaxParams];
  long long sy, sz;
  int nx, ny, nz, zc;
  int tiles_x, tiles_y, nblocks, x0;
};

// hipRTC options: the target, no contraction (each operation of the body is
// rounded on its own), no packed FP32 instructions.
int rtc_compile(const std::string& src, std::vector<char>* code) {
  hiprtcProgram prog = nullptr;
  if (hiprtcCreateProgram(&prog, src.c_str(), "ms_jit.hip", 0, nullptr, nullptr) !=
      HIPRTC_SUCCESS)
    return set_error(MS_EHIP, "ms_jit_compile: hiprtcCreateProgram failed");
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-ffp-contract=off", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof *opts), opts);
  int rc = MS_OK;
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    std::string log;
    if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
      log.resize(n);
      (void)hiprtcGetProgramLog(prog, &log[0]);
      if (log.size() > 600) log.resize(600);
    }
    rc = set_error(MS_EHIP, "ms_jit_compile: hipRTC: %s %s", hiprtcGetErrorString(r),
                   log.c_str());
  } else {
    size_t n = 0;
    if (hiprtcGetCodeSize(prog, &n) != HIPRTC_SUCCESS || n == 0) {
      rc = set_error(MS_EHIP, "ms_jit_compile: no code object");
    } else {
      code->resize(n);
      if (hiprtcGetCode(prog, code->data()) != HIPRTC_SUCCESS)
        rc = set_error(MS_EHIP, "ms_jit_compile: hiprtcGetCode failed");
    }
  }
  (void)hiprtcDestroyProgram(&prog);
  return rc;
}

}  // namespace
}  // namespace ms

namespace ms {
namespace {
struct JitModule {
  hipModule_t module;
  hipFunction_t scalar, vector;
};
}  // namespace
}  // namespace ms

struct ms_jit_stencil {
  ms::Program prog;
  int dtype = MS_F64;
  std::string source;
  std::vector<char> code;
  std::mutex mu;                         // guards `mods`
  std::map<int, ms::JitModule> mods;     // per device
};

using namespace ms;

extern "C" int ms_jit_compile(const char* program, int dtype, ms_jit_stencil** out) {
  clear_error();
  if (!program || !out) return set_error(MS_EINVAL, "ms_jit_compile: program and out required");
  *out = nullptr;
  if (dtype != MS_F64 && dtype != MS_F32)
    return set_error(MS_EUNSUPPORTED, "ms_jit_compile: dtype %d", dtype);
  if (std::strlen(program) > kJitMaxSource)
    return set_error(MS_EINVAL, "ms_jit_compile: program longer than %zu bytes", kJitMaxSource);
  try {
    Program p = Parser(program).run();
    std::string src = generate(p, dtype);
    std::vector<char> code;
    if (int rc = rtc_compile(src, &code)) return rc;
    auto* st = new ms_jit_stencil;
    st->prog = std::move(p);
    st->dtype = dtype;
    st->source = std::move(src);
    st->code = std::move(code);
    *out = st;
    return MS_OK;
  } catch (const ParseError& e) {
    return set_error(MS_EINVAL, "ms_jit_compile: %s", e.msg.c_str());
  } catch (const std::exception& e) {
    return set_error(MS_EINVAL, "ms_jit_compile: %s", e.what());
  }
}

extern "C" void ms_jit_free(ms_jit_stencil* st) {
  if (!st) return;
  int cur = -1;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  for (auto& kv : st->mods) {
    if (hipSetDevice(kv.first) == hipSuccess) (void)hipModuleUnload(kv.second.module);
  }
  if (have) (void)hipSetDevice(cur);
  delete st;
}

extern "C" const char* ms_jit_source(const ms_jit_stencil* st) {
  return st ? st->source.c_str() : nullptr;
}

extern "C" int ms_jit_signature(const ms_jit_stencil* st, int* n_fields, int* n_params,
                                int* n_profiles, int* n_outputs) {
  clear_error();
  if (!st) return set_error(MS_EINVAL, "ms_jit_signature: NULL program");
  if (n_fields) *n_fields = (int)st->prog.fields.size();
  if (n_params) *n_params = (int)st->prog.params.size();
  if (n_profiles) *n_profiles = (int)st->prog.profiles.size();
  if (n_outputs) *n_outputs = (int)st->prog.out_names.size();
  return MS_OK;
}

extern "C" const char* ms_jit_name(const ms_jit_stencil* st, int kind, int index) {
  if (!st || index < 0) return nullptr;
  const std::vector<std::string>* v = kind == MS_JIT_FIELD     ? &st->prog.fields
                                      : kind == MS_JIT_PARAM   ? &st->prog.params
                                      : kind == MS_JIT_PROFILE ? &st->prog.profiles
                                      : kind == MS_JIT_OUTPUT  ? &st->prog.out_names
                                                               : nullptr;
  if (!v || (size_t)index >= v->size()) return nullptr;
  return (*v)[index].c_str();
}

namespace {

// The module's two kernels on the current device (loaded on first use).
int jit_functions(ms_jit_stencil* st, hipFunction_t* scalar, hipFunction_t* vector) {
  int dev = 0;
  MS_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(st->mu);
  auto it = st->mods.find(dev);
  if (it == st->mods.end()) {
    JitModule jm{};
    MS_HIP_TRY(hipModuleLoadData(&jm.module, st->code.data()));
    hipError_t e = hipModuleGetFunction(&jm.scalar, jm.module, "ms_jit_kernel_s");
    if (e == hipSuccess) e = hipModuleGetFunction(&jm.vector, jm.module, "ms_jit_kernel_v");
    if (e != hipSuccess) {
      (void)hipModuleUnload(jm.module);
      return set_error(MS_EHIP, "ms_jit_apply: kernel not found: %s", hipGetErrorString(e));
    }
    it = st->mods.emplace(dev, jm).first;
  }
  *scalar = it->second.scalar;
  *vector = it->second.vector;
  return MS_OK;
}

// z split so that one launch has about `target` blocks (MS_JIT_BLOCKS
// overrides), marches of at least 8 levels. Measured at 512^3: the vector
// kernel is fastest near 256 blocks (one per CU, long marches), the scalar
// one near 4096.
template <typename T>
int jit_geometry(JitArgs<T>& a, int nz, int64_t target) {
  const char* ev = getenv("MS_JIT_BLOCKS");
  const int64_t want = ev && atoi(ev) > 0 ? atoi(ev) : target;
  const int64_t t2 = (int64_t)a.tiles_x * a.tiles_y;
  int64_t chunks = (want + t2 - 1) / t2;
  const int64_t max_chunks = (nz + 7) / 8;
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  a.zc = (int)((nz + chunks - 1) / chunks);
  chunks = (nz + a.zc - 1) / a.zc;
  const int64_t nb = t2 * chunks;
  if (nb > 0x7fffffff) return set_error(MS_EUNSUPPORTED, "ms_jit_apply: grid too large");
  a.nblocks = (int)nb;
  return MS_OK;
}

template <typename T>
int jit_launch(ms_jit_stencil* st, const ms_grid& g, const void* const* fields,
               const double* params, const void* const* profiles, void* const* outputs,
               hipStream_t s) {
  const Program& p = st->prog;
  JitArgs<T> a{};
  std::vector<const void*> ptrs;
  for (size_t q = 0; q < p.fields.size(); ++q) {
    a.in[q] = static_cast<const T*>(fields[q]);
    ptrs.push_back(fields[q]);
  }
  for (size_t q = 0; q < p.out_names.size(); ++q) {
    a.out[q] = static_cast<T*>(outputs[q]);
    ptrs.push_back(outputs[q]);
  }
  for (size_t q = 0; q < p.profiles.size(); ++q) a.prof[q] = static_cast<const T*>(profiles[q]);
  for (size_t q = 0; q < p.params.size(); ++q) a.prm[q] = (T)params[q];
  a.sy = g.sy;
  a.sz = g.sz;
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.tiles_y = (g.ny + 3) / 4;
  hipFunction_t fs = nullptr, fv = nullptr;
  if (int rc = jit_functions(st, &fs, &fv)) return rc;
  // Whole 64V-column tiles go to the vector kernel when every field is
  // aligned to V cells; the remaining columns to the scalar kernel.
  const int vmax = 16 / (int)sizeof(T);
  const int vec = vec_alignment(g, sizeof(T) == 8 ? MS_F64 : MS_F32, ptrs.data(),
                                (int)ptrs.size());
  const char* ev = getenv("MS_JIT_SCALAR");
  const int full = vec == vmax && !(ev && atoi(ev) > 0) ? g.nx / (64 * vmax) : 0;
  void* kargs[] = {&a};
  if (full > 0) {
    a.tiles_x = full;
    a.tiles_y = (g.ny + 4 * kJitVecRows - 1) / (4 * kJitVecRows);
    a.x0 = 0;
    if (int rc = jit_geometry(a, g.nz, 256)) return rc;
    MS_HIP_TRY(hipModuleLaunchKernel(fv, (unsigned)a.nblocks, 1, 1, 256, 1, 1, 0, s, kargs,
                                     nullptr));
  }
  a.x0 = full * 64 * vmax;
  if (a.x0 < g.nx) {
    a.tiles_x = (g.nx - a.x0 + 63) / 64;
    a.tiles_y = (g.ny + 3) / 4;
    if (int rc = jit_geometry(a, g.nz, 4096)) return rc;
    MS_HIP_TRY(hipModuleLaunchKernel(fs, (unsigned)a.nblocks, 1, 1, 256, 1, 1, 0, s, kargs,
                                     nullptr));
  }
  return MS_OK;
}

}  // namespace

extern "C" int ms_jit_apply(ms_jit_stencil* st, const ms_grid* g, const void* const* fields,
                            int n_fields, const double* params, int n_params,
                            const void* const* profiles, int n_profiles, void* const* outputs,
                            int n_outputs, void* stream) {
  clear_error();
  if (!st) return set_error(MS_EINVAL, "ms_jit_apply: NULL program");
  if (int rc = check_grid(g, "ms_jit_apply")) return rc;
  const Program& p = st->prog;
  if (n_fields != (int)p.fields.size() || n_params != (int)p.params.size() ||
      n_profiles != (int)p.profiles.size() || n_outputs != (int)p.out_names.size())
    return set_error(MS_EINVAL,
                     "ms_jit_apply: the program takes %zu fields, %zu params, %zu profiles, "
                     "%zu outputs",
                     p.fields.size(), p.params.size(), p.profiles.size(), p.out_names.size());
  if ((n_fields && !fields) || (n_params && !params) || (n_profiles && !profiles) || !outputs)
    return set_error(MS_EINVAL, "ms_jit_apply: missing argument array");
  for (int q = 0; q < n_fields; ++q)
    if (!fields[q]) return set_error(MS_EINVAL, "ms_jit_apply: field %d is NULL", q);
  for (int q = 0; q < n_profiles; ++q)
    if (!profiles[q]) return set_error(MS_EINVAL, "ms_jit_apply: profile %d is NULL", q);
  const size_t esz = st->dtype == MS_F64 ? 8 : 4;
  const size_t fbytes = (size_t)field_span(*g) * esz, pbytes = (size_t)g->nz * esz;
  for (int r = 0; r < n_outputs; ++r) {
    if (!outputs[r]) return set_error(MS_EINVAL, "ms_jit_apply: output %d is NULL", r);
    for (int q = 0; q < n_fields; ++q)
      if (overlaps(outputs[r], fbytes, fields[q], fbytes))
        return set_error(MS_EINVAL, "ms_jit_apply: output %d overlaps field %d", r, q);
    for (int q = 0; q < n_profiles; ++q)
      if (overlaps(outputs[r], fbytes, profiles[q], pbytes))
        return set_error(MS_EINVAL, "ms_jit_apply: output %d overlaps profile %d", r, q);
    for (int q = 0; q < r; ++q)
      if (overlaps(outputs[r], fbytes, outputs[q], fbytes))
        return set_error(MS_EINVAL, "ms_jit_apply: outputs %d and %d overlap", q, r);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (st->dtype == MS_F64) return jit_launch<double>(st, *g, fields, params, profiles, outputs, s);
  return jit_launch<float>(st, *g, fields, params, profiles, outputs, s);
}
