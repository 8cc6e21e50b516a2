// program.cpp -- layered evaluation of linear binary Datalog programs.
//
// A program is parsed, its predicates are split into strongly connected
// components of the dependency graph with Tarjan's algorithm and taken in
// dependency order as layers (Sec. 5).  Clause bodies are chains from the
// head's first argument to its second; along a chain a conjunction is a
// product of relation matrices, an atom written with swapped arguments is
// the transposed matrix, and a negated atom of a lower layer is the
// complement 1 - R (Sec. 5, Sec. 8).  Each clause of a layer is therefore
//   R_h  <-  P R_j^o S      (one atom of the layer, Sec. 5 linearity)
// or a constant term, and a layer is the system R_h = min1(A_h + sum P R^o S).
// A layer is evaluated by
//   * the Boolean iteration of its series from R = 0 (every form; int8
//     products on the matrix cores, Jacobi order, stop at the first
//     repeat), or by an epsilon form (Sec. 6):
//   * tail recursive layers (every recursive atom at the right end of its
//     chain, or every one at the left end, which is the same after
//     transposition) as one stacked fp64 linear system
//     X_h = eps_h (A_h + sum_j B_hj X_j), solved by block elimination -- the
//     layer-wide form of substituting one head's solution into the others;
//   * a single two-sided or transposed clause as the discrete Stein
//     equation X = eps (Q + B X C) by fp64 doubling; the transposed clause
//     R = A + P R^T S is first substituted into itself (Sec. 6.2), giving
//     Q = A + P A^T S, B = P S^T, C = P^T S.
// Thresholding the epsilon solutions at > 0 gives the layer's least model
// (Sec. 5, the theorem on layered evaluation; exact up to fp64 underflow).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/dl.h"
#include "common.h"
#include "ctx.h"
#include "eps_solve.h"

using namespace dl;

namespace {

int perr(int status, const std::string& msg) {
  set_last_error(msg);
  return status;
}

#define P_HIP(expr)                                                                       \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return perr(DL_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define P_RC(expr)          \
  do {                      \
    int rc_ = (expr);       \
    if (rc_) return rc_;    \
  } while (0)

// ----------------------------------------------------------------- syntax
struct SAtom {
  std::string pred, a, b;
  bool neg = false;
  int line = 0;
};
struct SClause {
  SAtom head;
  std::vector<SAtom> body;
};

bool is_pred_name(const std::string& s) { return !s.empty() && std::islower((unsigned char)s[0]); }
bool is_var_name(const std::string& s) { return !s.empty() && std::isupper((unsigned char)s[0]); }

struct Lexer {
  const char* p;
  int line = 1;
  std::string tok;
  bool next() {
    for (;;) {
      while (*p && std::isspace((unsigned char)*p)) {
        if (*p == '\n') ++line;
        ++p;
      }
      if (*p == '%') {
        while (*p && *p != '\n') ++p;
        continue;
      }
      break;
    }
    if (!*p) {
      tok.clear();
      return false;
    }
    if (std::isalnum((unsigned char)*p) || *p == '_') {
      const char* q = p;
      while (std::isalnum((unsigned char)*q) || *q == '_') ++q;
      tok.assign(p, q);
      p = q;
    } else if (p[0] == ':' && p[1] == '-') {
      tok = ":-";
      p += 2;
    } else if (p[0] == '\\' && p[1] == '+') {
      tok = "not";
      p += 2;
    } else {
      tok.assign(p, 1);
      ++p;
    }
    return true;
  }
};

int parse(const char* text, std::vector<SClause>* out) {
  Lexer lx{text};
  auto where = [&]() { return "line " + std::to_string(lx.line) + ": "; };
  bool more = lx.next();
  auto expect = [&](const char* t) -> int {
    if (!more || lx.tok != t) return perr(DL_EINVAL, where() + "expected '" + t + "'");
    more = lx.next();
    return DL_OK;
  };
  auto atom = [&](SAtom* a) -> int {
    if (more && lx.tok == "not") {
      a->neg = true;
      more = lx.next();
    }
    if (!more || !is_pred_name(lx.tok)) return perr(DL_EINVAL, where() + "expected a predicate name");
    a->pred = lx.tok;
    a->line = lx.line;
    more = lx.next();
    P_RC(expect("("));
    if (!more || !is_var_name(lx.tok))
      return perr(DL_EINVAL, where() + "arguments must be variables (capitalised names)");
    a->a = lx.tok;
    more = lx.next();
    P_RC(expect(","));
    if (!more || !is_var_name(lx.tok))
      return perr(DL_EINVAL, where() + "arguments must be variables (capitalised names)");
    a->b = lx.tok;
    more = lx.next();
    if (more && lx.tok == ",") return perr(DL_EINVAL, where() + "predicates are binary");
    return expect(")");
  };
  while (more) {
    SClause c;
    P_RC(atom(&c.head));
    if (c.head.neg) return perr(DL_EINVAL, where() + "negated head");
    if (!more || lx.tok != ":-") return perr(DL_EINVAL, where() + "facts are given as bound relations, not clauses");
    more = lx.next();
    for (;;) {
      SAtom a;
      P_RC(atom(&a));
      c.body.push_back(a);
      if (more && lx.tok == ",") {
        more = lx.next();
        continue;
      }
      break;
    }
    P_RC(expect("."));
    out->push_back(std::move(c));
  }
  if (out->empty()) return perr(DL_EINVAL, "empty program");
  return DL_OK;
}

// ----------------------------------------------------------------- semantics
enum Kind { K_GIVEN = 0, K_DEFINED = 1, K_EQ = 2 };

struct Factor {
  int pred = -1;
  bool trans = false;  // atom read against its written argument order
  bool neg = false;
};

struct Term {
  int head = -1;                // predicate index of the head
  std::vector<Factor> factors;  // the whole chain
  int rec = -1;                 // position of the atom of the head's layer, -1 = none
};

struct Mat {
  int8_t* M = nullptr;  // row-major
  int8_t* T = nullptr;  // its transpose
  bool ident = false;   // the identity (no storage)
};

}  // namespace

struct dl_program {
  dl_ctx* ctx = nullptr;
  std::vector<std::string> names;
  std::vector<int> kind;
  std::vector<int> layer_of;
  std::vector<std::vector<int>> layers;  // predicate indices per layer, dependency order
  std::vector<Term> terms;
  // per layer after a run
  std::vector<int> form, method_used, iters;
  // bindings
  int64_t n = -1;
  std::vector<const uint8_t*> bound;
  std::vector<int64_t> bound_ld;
  // device state
  int64_t Np = 0;
  bool ran = false;
  std::vector<Mat> val, comp;
  std::vector<void*> keep;  // allocations holding results
  size_t bytes = 0;
  unsigned long long* dcnt = nullptr;  // device counters
  unsigned long long* hcnt = nullptr;  // pinned mirror
};

namespace {

int pred_index(dl_program* g, const std::string& name) {
  for (size_t i = 0; i < g->names.size(); ++i)
    if (g->names[i] == name) return (int)i;
  return -1;
}

int intern(dl_program* g, const std::string& name) {
  int i = pred_index(g, name);
  if (i >= 0) return i;
  g->names.push_back(name);
  g->kind.push_back(name == "eq" ? K_EQ : K_GIVEN);
  return (int)g->names.size() - 1;
}

// The body as a chain from the head's first variable to its second.
int chain(const SClause& c, const std::vector<int>& preds, std::vector<Factor>* out) {
  const std::string where = "line " + std::to_string(c.head.line) + ": ";
  const std::string x = c.head.a, z = c.head.b;
  if (x == z) return perr(DL_EUNSUPPORTED, where + "head arguments must be two different variables");
  std::map<std::string, int> deg;
  for (const SAtom& a : c.body) {
    if (a.a == a.b) return perr(DL_EUNSUPPORTED, where + "atom with a repeated variable is not a chain link");
    ++deg[a.a];
    ++deg[a.b];
  }
  for (auto& kv : deg) {
    const int want = (kv.first == x || kv.first == z) ? 1 : 2;
    if (kv.second != want)
      return perr(DL_EUNSUPPORTED, where + "body is not a chain from the first head argument to the second");
  }
  if (!deg.count(x) || !deg.count(z))
    return perr(DL_EUNSUPPORTED, where + "body is not a chain from the first head argument to the second");
  std::vector<bool> used(c.body.size(), false);
  std::string cur = x;
  for (size_t step = 0; step < c.body.size(); ++step) {
    int pick = -1;
    for (size_t k = 0; k < c.body.size(); ++k)
      if (!used[k] && (c.body[k].a == cur || c.body[k].b == cur)) {
        pick = (int)k;
        break;
      }
    if (pick < 0) return perr(DL_EUNSUPPORTED, where + "body is not a chain from the first head argument to the second");
    used[pick] = true;
    const SAtom& a = c.body[pick];
    Factor f;
    f.pred = preds[pick];
    f.neg = a.neg;
    f.trans = a.a != cur;
    cur = f.trans ? a.a : a.b;
    out->push_back(f);
  }
  if (cur != z) return perr(DL_EUNSUPPORTED, where + "body is not a chain from the first head argument to the second");
  return DL_OK;
}

// Tarjan's strongly connected components over the defined predicates; the
// components come out with every component after the ones it depends on.
void tarjan(int m, const std::vector<std::vector<int>>& adj, std::vector<std::vector<int>>* comps) {
  std::vector<int> index(m, -1), low(m, 0), stack;
  std::vector<bool> on(m, false);
  int counter = 0;
  std::function<void(int)> visit = [&](int v) {
    index[v] = low[v] = counter++;
    stack.push_back(v);
    on[v] = true;
    for (int w : adj[v]) {
      if (index[w] < 0) {
        visit(w);
        low[v] = std::min(low[v], low[w]);
      } else if (on[w]) {
        low[v] = std::min(low[v], index[w]);
      }
    }
    if (low[v] == index[v]) {
      std::vector<int> comp;
      int w;
      do {
        w = stack.back();
        stack.pop_back();
        on[w] = false;
        comp.push_back(w);
      } while (w != v);
      std::sort(comp.begin(), comp.end());
      comps->push_back(comp);
    }
  };
  for (int v = 0; v < m; ++v)
    if (index[v] < 0) visit(v);
}

int analyse(dl_program* g, const std::vector<SClause>& cs) {
  std::vector<std::vector<int>> body_preds;
  for (const SClause& c : cs) {
    if (c.head.pred == "eq") return perr(DL_EINVAL, "line " + std::to_string(c.head.line) + ": eq is built in");
    const int h = intern(g, c.head.pred);
    g->kind[h] = K_DEFINED;
    std::vector<int> bp;
    for (const SAtom& a : c.body) bp.push_back(intern(g, a.pred));
    body_preds.push_back(bp);
  }
  const int m = (int)g->names.size();
  std::vector<std::vector<int>> adj(m);
  for (size_t k = 0; k < cs.size(); ++k) {
    const int h = pred_index(g, cs[k].head.pred);
    for (int p : body_preds[k])
      if (g->kind[p] == K_DEFINED) adj[h].push_back(p);
  }
  std::vector<std::vector<int>> comps;
  tarjan(m, adj, &comps);
  g->layer_of.assign(m, -1);
  for (auto& comp : comps) {
    if (g->kind[comp[0]] != K_DEFINED) continue;  // given relations and eq are not layers
    for (int p : comp) g->layer_of[p] = (int)g->layers.size();
    g->layers.push_back(comp);
  }
  for (size_t k = 0; k < cs.size(); ++k) {
    const std::string where = "line " + std::to_string(cs[k].head.line) + ": ";
    Term t;
    t.head = pred_index(g, cs[k].head.pred);
    P_RC(chain(cs[k], body_preds[k], &t.factors));
    const int L = g->layer_of[t.head];
    for (size_t i = 0; i < t.factors.size(); ++i) {
      const Factor& f = t.factors[i];
      if (g->kind[f.pred] != K_DEFINED || g->layer_of[f.pred] != L) continue;
      if (f.neg)
        return perr(DL_EUNSUPPORTED, where + "negation of " + g->names[f.pred] +
                                         " inside its own layer: the program is not stratified");
      if (t.rec >= 0)
        return perr(DL_EUNSUPPORTED, where + "two atoms of the head's layer in one body: the program is not linear");
      t.rec = (int)i;
    }
    g->terms.push_back(t);
  }
  g->bound.assign(m, nullptr);
  g->bound_ld.assign(m, 0);
  return DL_OK;
}

// ----------------------------------------------------------------- device evaluation
enum Form { F_NONREC = 0, F_RIGHT_TAIL = 1, F_LEFT_TAIL = 2, F_TWO_SIDED = 3, F_GENERAL = 4 };

struct Runner {
  dl_program* g;
  hipStream_t s;
  int64_t n, Np;
  int cfg;
  TileCfg tc;
  std::vector<void*> temps;  // freed after each layer
  std::vector<EventPair> evs;  // product launches, when the context times kernels

  int alloc(int8_t** p, bool keep) {
    const size_t b = (size_t)Np * Np;
    if (g->ctx->budget && g->bytes + b > g->ctx->budget)
      return perr(DL_ENOMEM, "program matrices exceed the workspace budget");
    void* q = nullptr;
    if (hipMalloc(&q, b) != hipSuccess) {
      (void)hipGetLastError();
      return perr(DL_ENOMEM, "hipMalloc of a program matrix failed");
    }
    g->bytes += b;
    (keep ? g->keep : temps).push_back(q);
    *p = (int8_t*)q;
    return DL_OK;
  }
  int alloc_mat(Mat* m, bool keep) {
    P_RC(alloc(&m->M, keep));
    return alloc(&m->T, keep);
  }
  void free_temps() {
    const size_t b = (size_t)Np * Np;
    if (!temps.empty()) (void)hipStreamSynchronize(s);  // launches may still read them
    for (void* q : temps) {
      (void)hipFree(q);
      g->bytes -= b;
    }
    temps.clear();
  }
  // Moves a temporary allocation into the kept set (a layer result).
  void keep_ptr(void* q) {
    auto it = std::find(temps.begin(), temps.end(), q);
    if (it != temps.end()) {
      temps.erase(it);
      g->keep.push_back(q);
    }
  }

  // out = [add + X Y^T != 0] (+ I), int8; counts into *cnt when set.
  int nt(const int8_t* X, const int8_t* Y, const int8_t* add, int8_t* out, int8_t* outT, unsigned long long* cnt) {
    NTParams p{};
    p.X = X;
    p.Y = Y;
    p.ld = Np;
    p.Np = (int)Np;
    p.add = add;
    p.add_identity = 0;
    p.n_valid = (int)n;
    p.out = out;
    p.outT = outT;
    p.ones = cnt;
    p.count = cnt ? 1 : 0;
    p.conv = nullptr;
    p.step = 0;
    p.check = 0;
    p.tiles_m = (int)(Np / tc.bm);
    p.tiles_n = (int)(Np / tc.bn);
    EventPair ev{nullptr, nullptr};
    if (g->ctx->timing && hipEventCreate(&ev.a) == hipSuccess && hipEventCreate(&ev.b) == hipSuccess)
      (void)hipEventRecord(ev.a, s);
    P_HIP(launch_nt_step(P_I8, cfg, p, s));
    if (ev.a && ev.b) {
      (void)hipEventRecord(ev.b, s);
      evs.push_back(ev);
    }
    return DL_OK;
  }
  // Adds the recorded product launches to the context's class-0 statistics
  // (after the stream has been synchronised) and frees the events.
  void collect_events(bool ok) {
    for (auto& e : evs) {
      float t = 0.f;
      if (ok && hipEventElapsedTime(&t, e.a, e.b) == hipSuccess) {
        g->ctx->ms[0] += t;
        g->ctx->launches[0] += 1;
      }
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    evs.clear();
  }

  Mat view(const Factor& f) {
    Mat m = (f.neg ? g->comp : g->val)[f.pred];
    if (f.trans) std::swap(m.M, m.T);
    return m;
  }

  // Ensures the complement of a predicate used negated exists.
  int need_comp(int p) {
    if (g->comp[p].M) return DL_OK;
    Mat c;
    P_RC(alloc_mat(&c, true));
    P_HIP(launch_bytes_op(g->val[p].M, nullptr, 0, 1, (int)n, (int)Np, c.M, nullptr, nullptr, s));
    P_HIP(launch_bytes_op(g->val[p].T, nullptr, 0, 1, (int)n, (int)Np, c.T, nullptr, nullptr, s));
    g->comp[p] = c;
    return DL_OK;
  }

  // L * R as a 0/1 matrix with both orientations (identity operands pass through).
  int mul(const Mat& L, const Mat& R, Mat* out) {
    if (L.ident) {
      *out = R;
      return DL_OK;
    }
    if (R.ident) {
      *out = L;
      return DL_OK;
    }
    P_RC(alloc_mat(out, false));
    return nt(L.M, R.T, nullptr, out->M, out->T, nullptr);
  }

  Mat transposed(const Mat& m) {
    Mat t = m;
    std::swap(t.M, t.T);
    return t;
  }

  // Product of factors [b, e) of a chain; identity for an empty range.
  int product(const std::vector<Factor>& fs, size_t b, size_t e, Mat* out) {
    Mat acc;
    acc.ident = true;
    for (size_t i = b; i < e; ++i) {
      const Factor& f = fs[i];
      if (g->kind[f.pred] == K_EQ && !f.neg) continue;  // I X = X
      if (f.neg) P_RC(need_comp(f.pred));
      Mat nx;
      P_RC(mul(acc, view(f), &nx));
      acc = nx;
    }
    *out = acc;
    return DL_OK;
  }

  // Row-sum norm ||M||_inf of a 0/1 matrix.
  int norm_inf(const int8_t* M, int* out) {
    P_HIP(hipMemsetAsync(g->ctx->dscratch, 0, sizeof(int), s));
    P_HIP(launch_row_max((const uint8_t*)M, Np, (int)n, g->ctx->dscratch, s));
    P_HIP(hipMemcpyAsync(g->ctx->h_conv + 1, g->ctx->dscratch, sizeof(int), hipMemcpyDeviceToHost, s));
    P_HIP(hipStreamSynchronize(s));
    *out = g->ctx->h_conv[1];
    return DL_OK;
  }

  int ident_mat(Mat* out) {
    P_RC(alloc_mat(out, false));
    P_HIP(launch_bytes_op(nullptr, nullptr, 1, 0, (int)n, (int)Np, out->M, out->T, nullptr, s));
    return DL_OK;
  }

  int run_layer(int L, int method);
  int iterate(int L, const std::vector<int>& heads, const std::vector<Mat>& A, const std::vector<const Term*>& rec);
};

int Runner::run_layer(int L, int method) {
  const std::vector<int>& heads = g->layers[L];
  const int M = (int)heads.size();
  auto local = [&](int p) { return (int)(std::find(heads.begin(), heads.end(), p) - heads.begin()); };
  // constant parts A_h (both orientations) and the recursive terms
  std::vector<Mat> A(M);
  std::vector<const Term*> rec;
  for (int h = 0; h < M; ++h) {
    P_RC(alloc_mat(&A[h], false));
    P_HIP(hipMemsetAsync(A[h].M, 0, (size_t)Np * Np, s));
  }
  for (const Term& t : g->terms) {
    if (g->layer_of[t.head] != L) continue;
    if (t.rec >= 0) {
      rec.push_back(&t);
      continue;
    }
    Mat c;
    P_RC(product(t.factors, 0, t.factors.size(), &c));
    const int h = local(t.head);
    P_HIP(launch_bytes_op(A[h].M, c.ident ? nullptr : c.M, c.ident ? 1 : 0, 0, (int)n, (int)Np, A[h].M, nullptr,
                          nullptr, s));
  }
  P_HIP(hipMemsetAsync(g->dcnt, 0, (size_t)M * sizeof(unsigned long long), s));
  for (int h = 0; h < M; ++h)
    P_HIP(launch_bytes_op(A[h].M, nullptr, 0, 0, (int)n, (int)Np, nullptr, A[h].T, g->dcnt + h, s));

  // form of the layer
  int form = F_GENERAL;
  if (rec.empty()) {
    form = F_NONREC;
  } else {
    bool right = true, left = true;
    for (const Term* t : rec) {
      const Factor& r = t->factors[t->rec];
      if (r.trans || t->rec + 1 != (int)t->factors.size()) right = false;
      if (r.trans || t->rec != 0) left = false;
    }
    if (right && M <= kMaxStack)
      form = F_RIGHT_TAIL;
    else if (left && M <= kMaxStack)
      form = F_LEFT_TAIL;
    else if (M == 1 && rec.size() == 1)
      form = F_TWO_SIDED;
  }
  g->form[L] = form;

  if (form == F_NONREC) {
    for (int h = 0; h < M; ++h) {
      g->val[heads[h]] = A[h];
      keep_ptr(A[h].M);
      keep_ptr(A[h].T);
    }
    // the series R^(1) = A, R^(2) = A: the confirming application is the
    // second one unless A is empty
    P_HIP(hipMemcpyAsync(g->hcnt, g->dcnt, (size_t)M * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    P_HIP(hipStreamSynchronize(s));
    unsigned long long ones = 0;
    for (int h = 0; h < M; ++h) ones += g->hcnt[h];
    g->method_used[L] = DL_EVAL_ITERATION;
    g->iters[L] = ones ? 2 : 1;
    return DL_OK;
  }
  if (method == DL_EVAL_ITERATION || form == F_GENERAL) {
    g->method_used[L] = DL_EVAL_ITERATION;
    return iterate(L, heads, A, rec);
  }
  g->method_used[L] = DL_EVAL_MATRIX;
  std::string err;
  if (form == F_RIGHT_TAIL || form == F_LEFT_TAIL) {
    // X_h = eps_h (A_h + sum_j B_hj X_j); the left form is solved for R^T
    const bool lt = form == F_LEFT_TAIL;
    StackDesc d;
    d.M = M;
    d.Np = (int)Np;
    std::vector<std::vector<Mat>> B(M, std::vector<Mat>(M));
    Mat I;
    for (const Term* t : rec) {
      Mat part;
      if (lt)
        P_RC(product(t->factors, 1, t->factors.size(), &part));  // S, used as S^T
      else
        P_RC(product(t->factors, 0, (size_t)t->rec, &part));  // P
      if (part.ident) {
        if (!I.M) P_RC(ident_mat(&I));
        part = I;
      }
      if (lt) part = transposed(part);
      const int h = local(t->head), j = local(t->factors[t->rec].pred);
      Mat& b = B[h][j];
      if (!b.M) {
        b = part;
      } else {
        Mat o;
        P_RC(alloc(&o.M, false));
        P_HIP(launch_bytes_op(b.M, part.M, 0, 0, (int)n, (int)Np, o.M, nullptr, nullptr, s));
        b = o;
      }
    }
    for (int h = 0; h < M; ++h) {
      int sum = 0;
      for (int j = 0; j < M; ++j) {
        d.B[h][j] = B[h][j].M;
        if (B[h][j].M) {
          int nb = 0;
          P_RC(norm_inf(B[h][j].M, &nb));
          sum += nb;
        }
      }
      d.A[h] = lt ? A[h].T : A[h].M;
      d.eps[h] = 1.0 / (1.0 + (double)sum);
    }
    std::vector<Mat> R(M);
    for (int h = 0; h < M; ++h) {
      P_RC(alloc_mat(&R[h], true));
      d.R[h] = lt ? R[h].T : R[h].M;
    }
    d.cnt = nullptr;
    hipError_t e = stacked_solve(&g->ctx->eps, g->ctx->budget, d, s, &err);
    if (e == hipErrorOutOfMemory) return perr(DL_ENOMEM, err);
    if (e != hipSuccess) return perr(DL_EHIP, err + ": " + hipGetErrorString(e));
    for (int h = 0; h < M; ++h) {
      // the other orientation
      if (lt)
        P_HIP(launch_bytes_op(R[h].T, nullptr, 0, 0, (int)n, (int)Np, nullptr, R[h].M, nullptr, s));
      else
        P_HIP(launch_bytes_op(R[h].M, nullptr, 0, 0, (int)n, (int)Np, nullptr, R[h].T, nullptr, s));
      g->val[heads[h]] = R[h];
    }
    g->iters[L] = 0;
    return DL_OK;
  }
  // F_TWO_SIDED: one clause R = A + P R^o S
  const Term* t = rec[0];
  Mat P, S, Q, Bm, Cm;
  P_RC(product(t->factors, 0, (size_t)t->rec, &P));
  P_RC(product(t->factors, (size_t)t->rec + 1, t->factors.size(), &S));
  if (!t->factors[t->rec].trans) {
    Q = A[0];
    Bm = P;
    Cm = S;
  } else {
    // R = A + P (A^T + S^T R P^T) S = (A + P A^T S) + (P S^T) R (P^T S)
    Mat PAt, PAtS;
    P_RC(mul(P, transposed(A[0]), &PAt));
    P_RC(mul(PAt, S, &PAtS));
    P_RC(alloc_mat(&Q, false));
    P_HIP(launch_bytes_op(A[0].M, PAtS.M, 0, 0, (int)n, (int)Np, Q.M, Q.T, nullptr, s));
    P_RC(mul(P, transposed(S), &Bm));
    P_RC(mul(transposed(P), S, &Cm));
  }
  Mat I;
  if (Bm.ident || Cm.ident) P_RC(ident_mat(&I));
  if (Bm.ident) Bm = I;
  if (Cm.ident) Cm = I;
  int nb = 0, nc = 0;
  P_RC(norm_inf(Bm.M, &nb));
  P_RC(norm_inf(Cm.T, &nc));  // column sums of C
  const double eps = 1.0 / (1.0 + (double)nb * (double)nc);
  Mat R;
  P_RC(alloc_mat(&R, true));
  P_HIP(hipMemsetAsync(R.M, 0, (size_t)Np * Np, s));
  int32_t dbl = 0;
  hipError_t e = two_sided_solve(&g->ctx->eps, g->ctx->budget, n, (const uint8_t*)Q.M, Np, (const uint8_t*)Bm.M, Np,
                                 (const uint8_t*)Cm.M, Np, eps, nullptr, 0, nullptr, 0, R.M, Np, nullptr, 64, s, &dbl,
                                 (unsigned long long*)(g->ctx->dscratch + 8), g->ctx->h_ring, &err);
  if (e == hipErrorOutOfMemory) return perr(DL_ENOMEM, err);
  if (e == hipErrorNotReady) return perr(DL_ENOCONV, "doubling cap reached");
  if (e != hipSuccess) return perr(DL_EHIP, err + ": " + hipGetErrorString(e));
  P_HIP(launch_bytes_op(R.M, nullptr, 0, 0, (int)n, (int)Np, nullptr, R.T, nullptr, s));
  g->val[heads[0]] = R;
  g->iters[L] = dbl;
  return DL_OK;
}

// Boolean series of the layer: R^(0) = 0, R^(k+1)_h = min1(A_h + sum P R^o S)
// over R^(k), all heads at once; stops at the first k with R^(k) = R^(k-1).
int Runner::iterate(int L, const std::vector<int>& heads, const std::vector<Mat>& A,
                    const std::vector<const Term*>& rec) {
  const int M = (int)heads.size();
  auto local = [&](int p) { return (int)(std::find(heads.begin(), heads.end(), p) - heads.begin()); };
  struct Op {
    Mat P, S;
    int j;
    bool trans;
  };
  std::vector<std::vector<Op>> ops(M);
  for (const Term* t : rec) {
    Op o;
    P_RC(product(t->factors, 0, (size_t)t->rec, &o.P));
    P_RC(product(t->factors, (size_t)t->rec + 1, t->factors.size(), &o.S));
    o.j = local(t->factors[t->rec].pred);
    o.trans = t->factors[t->rec].trans;
    ops[local(t->head)].push_back(o);
  }
  std::vector<Mat> cur(M), nxt(M);
  for (int h = 0; h < M; ++h) {
    P_RC(alloc_mat(&cur[h], false));
    P_RC(alloc_mat(&nxt[h], false));
  }
  int8_t *acc[2], *tmp;
  P_RC(alloc(&acc[0], false));
  P_RC(alloc(&acc[1], false));
  P_RC(alloc(&tmp, false));
  // R^(1) = A
  P_HIP(hipMemsetAsync(g->dcnt, 0, (size_t)M * sizeof(unsigned long long), s));
  for (int h = 0; h < M; ++h)
    P_HIP(launch_bytes_op(A[h].M, nullptr, 0, 0, (int)n, (int)Np, cur[h].M, cur[h].T, g->dcnt + h, s));
  auto total = [&](int64_t* t) -> int {
    P_HIP(hipMemcpyAsync(g->hcnt, g->dcnt, (size_t)M * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    P_HIP(hipStreamSynchronize(s));
    int64_t sum = 0;
    for (int h = 0; h < M; ++h) sum += (int64_t)g->hcnt[h];
    *t = sum;
    return DL_OK;
  };
  int64_t prev = 0, now = 0;
  P_RC(total(&now));
  int k = 1;
  // every step before the repeat adds at least one of the M n^2 facts
  const int64_t cap = (int64_t)M * n * n + 2;
  while (now != prev && k < cap) {
    prev = now;
    ++k;
    P_HIP(hipMemsetAsync(g->dcnt, 0, (size_t)M * sizeof(unsigned long long), s));
    for (int h = 0; h < M; ++h) {
      // the head's current iterate stands in for its non-recursive part A[h]:
      // R^(k) = A + F(R^(k-1)) lies inside A + F(R^(k)) (F monotone, the
      // iterates grow) and contains A, so A + F(R^(k)) = R^(k) + F(R^(k));
      // for self-recursive terms it is also the product's left operand
      const int8_t* addp = cur[h].M;
      const size_t q = ops[h].size();
      for (size_t i = 0; i < q; ++i) {
        const Op& o = ops[h][i];
        const bool last = i + 1 == q;
        int8_t* dM = last ? nxt[h].M : acc[i & 1];
        int8_t* dT = last ? nxt[h].T : nullptr;
        unsigned long long* cnt = last ? g->dcnt + h : nullptr;
        Mat r = cur[o.j];
        if (o.trans) r = transposed(r);
        if (o.P.ident && o.S.ident) {
          P_HIP(launch_bytes_op(addp, r.M, 0, 0, (int)n, (int)Np, dM, dT, cnt, s));
        } else if (o.P.ident) {
          P_RC(nt(r.M, o.S.T, addp, dM, dT, cnt));
        } else if (o.S.ident) {
          P_RC(nt(o.P.M, r.T, addp, dM, dT, cnt));
        } else {
          P_RC(nt(o.P.M, r.T, nullptr, tmp, nullptr, nullptr));
          P_RC(nt(tmp, o.S.T, addp, dM, dT, cnt));
        }
        addp = dM;
      }
    }
    P_RC(total(&now));
    std::swap(cur, nxt);
  }
  if (now != prev) return perr(DL_ENOCONV, "layer iteration cap reached");
  for (int h = 0; h < M; ++h) {
    g->val[heads[h]] = cur[h];
    keep_ptr(cur[h].M);
    keep_ptr(cur[h].T);
  }
  g->iters[L] = k;
  return DL_OK;
}

void release(dl_program* g) {
  for (void* q : g->keep) (void)hipFree(q);
  g->keep.clear();
  g->bytes = 0;
  g->val.clear();
  g->comp.clear();
  g->ran = false;
}

}  // namespace

extern "C" {

int dl_program_create(dl_ctx* ctx, const char* text, dl_program** out) {
  if (!ctx || !text || !out) return perr(DL_EINVAL, "NULL argument");
  *out = nullptr;
  std::vector<SClause> cs;
  P_RC(parse(text, &cs));
  dl_program* g = new (std::nothrow) dl_program();
  if (!g) return perr(DL_ENOMEM, "host allocation failed");
  g->ctx = ctx;
  int rc = analyse(g, cs);
  if (rc) {
    delete g;
    return rc;
  }
  size_t widest = 1;
  for (auto& l : g->layers) widest = std::max(widest, l.size());
  if (hipSetDevice(ctx->device) != hipSuccess ||
      hipMalloc(&g->dcnt, widest * sizeof(unsigned long long)) != hipSuccess ||
      hipHostMalloc(&g->hcnt, widest * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    if (g->dcnt) (void)hipFree(g->dcnt);
    delete g;
    return perr(DL_ENOMEM, "counter allocation failed");
  }
  const size_t L = g->layers.size();
  g->form.assign(L, -1);
  g->method_used.assign(L, -1);
  g->iters.assign(L, 0);
  *out = g;
  return DL_OK;
}

int dl_program_destroy(dl_program* g) {
  if (!g) return DL_OK;
  (void)hipSetDevice(g->ctx->device);
  release(g);
  if (g->dcnt) (void)hipFree(g->dcnt);
  if (g->hcnt) (void)hipHostFree(g->hcnt);
  delete g;
  return DL_OK;
}

int dl_program_counts(dl_program* g, int32_t* n_predicates, int32_t* n_layers) {
  if (!g) return perr(DL_EINVAL, "program is NULL");
  if (n_predicates) *n_predicates = (int32_t)g->names.size();
  if (n_layers) *n_layers = (int32_t)g->layers.size();
  return DL_OK;
}

int dl_program_predicate(dl_program* g, int32_t index, const char** name, int32_t* kind, int32_t* layer) {
  if (!g || index < 0 || index >= (int32_t)g->names.size()) return perr(DL_EINVAL, "no such predicate");
  if (name) *name = g->names[index].c_str();
  if (kind) *kind = g->kind[index];
  if (layer) *layer = g->layer_of[index];
  return DL_OK;
}

int dl_program_bind(dl_program* g, const char* name, int64_t n, const uint8_t* M, int64_t ldm) {
  if (!g || !name) return perr(DL_EINVAL, "NULL argument");
  const int p = pred_index(g, name);
  if (p < 0) return perr(DL_EINVAL, std::string("the program does not use ") + name);
  if (g->kind[p] != K_GIVEN) return perr(DL_EINVAL, std::string(name) + " is not a given relation");
  if (n < 0 || n > (1 << 16)) return perr(DL_EINVAL, "bad n");
  if (n > 0 && (!M || ldm < n)) return perr(DL_EINVAL, "bad matrix");
  if (g->n >= 0 && n != g->n) {
    bool other = false;
    for (size_t i = 0; i < g->bound.size(); ++i) other |= (int)i != p && g->bound[i] != nullptr;
    if (other) return perr(DL_EINVAL, "all relations of a program share one n");
  }
  g->n = n;
  g->bound[p] = n > 0 ? M : (const uint8_t*)1;  // n = 0: nothing to read
  g->bound_ld[p] = ldm;
  return DL_OK;
}

int dl_program_run(dl_program* g, int method, void* stream) {
  if (!g) return perr(DL_EINVAL, "program is NULL");
  if (method != DL_EVAL_ITERATION && method != DL_EVAL_MATRIX) return perr(DL_EINVAL, "unknown method");
  for (size_t p = 0; p < g->names.size(); ++p)
    if (g->kind[p] == K_GIVEN && !g->bound[p])
      return perr(DL_EINVAL, "relation " + g->names[p] + " is neither defined nor bound");
  if (g->n < 0) g->n = 0;
  P_HIP(hipSetDevice(g->ctx->device));
  release(g);
  hipStream_t s = (hipStream_t)stream;
  Runner r{g, s, g->n, 0, 0, {}, {}};
  g->val.assign(g->names.size(), Mat());
  g->comp.assign(g->names.size(), Mat());
  if (g->n == 0) {
    for (size_t L = 0; L < g->layers.size(); ++L) {
      g->form[L] = -1;
      g->method_used[L] = method;
      g->iters[L] = 0;
    }
    g->ran = true;
    return DL_OK;
  }
  r.Np = padded_size_for(P_I8, g->n);
  g->Np = r.Np;
  r.cfg = pick_config(g->ctx, P_I8, r.Np);
  r.tc = nt_config(P_I8, r.cfg);
  int rc = DL_OK;
  for (size_t p = 0; p < g->names.size() && !rc; ++p) {
    if (g->kind[p] == K_GIVEN) {
      rc = r.alloc_mat(&g->val[p], true);
      if (!rc && launch_ingest(P_I8, g->bound[p], g->bound_ld[p], (int)g->n, (int)r.Np, g->val[p].M, g->val[p].T,
                               nullptr, nullptr, 0, nullptr, s) != hipSuccess)
        rc = perr(DL_EHIP, "ingest failed");
    } else if (g->kind[p] == K_EQ) {
      rc = r.alloc_mat(&g->val[p], true);
      if (!rc && launch_bytes_op(nullptr, nullptr, 1, 0, (int)g->n, (int)r.Np, g->val[p].M, g->val[p].T, nullptr,
                                 s) != hipSuccess)
        rc = perr(DL_EHIP, "identity failed");
    }
  }
  for (size_t L = 0; L < g->layers.size() && !rc; ++L) {
    rc = r.run_layer((int)L, method);
    r.free_temps();
  }
  r.free_temps();
  if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = perr(DL_EHIP, "stream synchronisation failed");
  r.collect_events(rc == DL_OK);
  if (rc) {
    release(g);
    return rc;
  }
  g->ran = true;
  return DL_OK;
}

int dl_program_layer(dl_program* g, int32_t layer, int32_t* n_heads, int32_t* heads, int32_t cap, int32_t* form,
                     int32_t* method_used, int32_t* iters) {
  if (!g || layer < 0 || layer >= (int32_t)g->layers.size()) return perr(DL_EINVAL, "no such layer");
  const auto& hs = g->layers[layer];
  if (n_heads) *n_heads = (int32_t)hs.size();
  for (int32_t i = 0; heads && i < cap && i < (int32_t)hs.size(); ++i) heads[i] = hs[i];
  if (form) *form = g->form[layer];
  if (method_used) *method_used = g->method_used[layer];
  if (iters) *iters = g->iters[layer];
  return DL_OK;
}

int dl_program_fetch(dl_program* g, const char* name, uint8_t* out, int64_t ldo, int64_t* ones, void* stream) {
  if (!g || !name) return perr(DL_EINVAL, "NULL argument");
  if (!g->ran) return perr(DL_EINVAL, "the program has not been run");
  const int p = pred_index(g, name);
  if (p < 0 || g->kind[p] != K_DEFINED) return perr(DL_EINVAL, std::string(name) + " is not defined by the program");
  if (g->n > 0 && (!out || ldo < g->n)) return perr(DL_EINVAL, "bad output matrix");
  if (g->n == 0) {
    if (ones) *ones = 0;
    return DL_OK;
  }
  P_HIP(hipSetDevice(g->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  P_HIP(launch_emit(P_I8, g->val[p].M, (int)g->Np, 0, (int)g->n, out, ldo, s));
  if (ones) {
    P_HIP(hipMemsetAsync(g->dcnt, 0, sizeof(unsigned long long), s));
    P_HIP(launch_bytes_op(g->val[p].M, nullptr, 0, 0, (int)g->n, (int)g->Np, nullptr, nullptr, g->dcnt, s));
    P_HIP(hipMemcpyAsync(g->hcnt, g->dcnt, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  }
  P_HIP(hipStreamSynchronize(s));
  if (ones) *ones = (int64_t)g->hcnt[0];
  return DL_OK;
}

}  // extern "C"
