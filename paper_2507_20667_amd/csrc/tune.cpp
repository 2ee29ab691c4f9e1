// The tuning table: launch choices measured on the GPU by the project's
// tuner (python -m paper_2507_20667_amd.tune) and read at plan load.
//
//   gemm rules  per (precision, form, ceil log2 of M, N and K): the tile
//               shape of the FP32 plane kernel and the number of k chunks;
//   tree rules  per plan fingerprint: queries per workgroup of the subtree
//               kernel, the size from which a per-query intermediate lives
//               in device memory, and the size limit of packed gate steps.
//
// The file is JSON: {"gemm": [{"prec": "fp32", "form": "3m", "lm": 10,
// "ln": 17, "lk": 10, "tile": 0, "ksplit": 1, ...}, ...], "tree":
// [{"fingerprint": "0123456789abcdef", "qw": 4, "spill": 512, "pack_nc": 64,
// ...}, ...]}; other keys are ignored.  It is found through TN_TUNE_FILE,
// else as tune.json beside libtn.so; "off" (or a missing file) means no
// rules: every choice is the built-in heuristic.
#include <dlfcn.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "tn_internal.h"

namespace tn {

namespace {

// A JSON value (only what the table needs: objects, arrays, strings, numbers).
struct JVal {
  enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
  double num = 0.0;
  std::string str;
  std::vector<JVal> arr;
  std::map<std::string, JVal> obj;
};

class JParser {
 public:
  explicit JParser(const std::string &s) : s_(s) {}
  bool parse(JVal &v) {
    if (!value(v)) return false;
    ws();
    return i_ == s_.size();
  }

 private:
  void ws() {
    while (i_ < s_.size() && isspace((unsigned char)s_[i_])) ++i_;
  }
  bool lit(const char *w) {
    const size_t n = strlen(w);
    if (s_.compare(i_, n, w) != 0) return false;
    i_ += n;
    return true;
  }
  bool string(std::string &out) {
    if (s_[i_] != '"') return false;
    ++i_;
    while (i_ < s_.size() && s_[i_] != '"') {
      if (s_[i_] == '\\') {
        if (++i_ >= s_.size()) return false;
        const char c = s_[i_];
        out += c == 'n' ? '\n' : c == 't' ? '\t' : c;  // \u escapes are not used here
      } else {
        out += s_[i_];
      }
      ++i_;
    }
    if (i_ >= s_.size()) return false;
    ++i_;
    return true;
  }
  bool value(JVal &v) {
    ws();
    if (i_ >= s_.size()) return false;
    const char c = s_[i_];
    if (c == '{') {
      v.kind = JVal::OBJ;
      ++i_;
      ws();
      if (i_ < s_.size() && s_[i_] == '}') {
        ++i_;
        return true;
      }
      while (true) {
        ws();
        std::string k;
        if (i_ >= s_.size() || !string(k)) return false;
        ws();
        if (i_ >= s_.size() || s_[i_] != ':') return false;
        ++i_;
        if (!value(v.obj[k])) return false;
        ws();
        if (i_ < s_.size() && s_[i_] == ',') {
          ++i_;
          continue;
        }
        if (i_ < s_.size() && s_[i_] == '}') {
          ++i_;
          return true;
        }
        return false;
      }
    }
    if (c == '[') {
      v.kind = JVal::ARR;
      ++i_;
      ws();
      if (i_ < s_.size() && s_[i_] == ']') {
        ++i_;
        return true;
      }
      while (true) {
        v.arr.emplace_back();
        if (!value(v.arr.back())) return false;
        ws();
        if (i_ < s_.size() && s_[i_] == ',') {
          ++i_;
          continue;
        }
        if (i_ < s_.size() && s_[i_] == ']') {
          ++i_;
          return true;
        }
        return false;
      }
    }
    if (c == '"') {
      v.kind = JVal::STR;
      return string(v.str);
    }
    if (lit("true")) {
      v.kind = JVal::BOOL;
      v.num = 1;
      return true;
    }
    if (lit("false")) {
      v.kind = JVal::BOOL;
      return true;
    }
    if (lit("null")) return true;
    const char *b = s_.c_str() + i_;
    char *e = nullptr;
    v.num = strtod(b, &e);
    if (e == b) return false;
    v.kind = JVal::NUM;
    i_ += (size_t)(e - b);
    return true;
  }
  const std::string &s_;
  size_t i_ = 0;
};

int jint(const JVal &o, const char *k, int dflt) {
  auto it = o.obj.find(k);
  return it != o.obj.end() && it->second.kind == JVal::NUM ? (int)it->second.num : dflt;
}
std::string jstr(const JVal &o, const char *k) {
  auto it = o.obj.find(k);
  return it != o.obj.end() && it->second.kind == JVal::STR ? it->second.str : std::string();
}

std::string default_path() {
  Dl_info info;
  if (dladdr((void *)&default_path, &info) && info.dli_fname) {
    std::string so = info.dli_fname;
    const size_t slash = so.rfind('/');
    return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tune.json";
  }
  return "tune.json";
}

}  // namespace

static TuneTable load_table() {
  TuneTable t;
  const char *env = getenv("TN_TUNE_FILE");
  if (env && (!*env || strcmp(env, "off") == 0)) return t;
  t.path = env ? env : default_path();
  std::ifstream f(t.path);
  if (!f) return t;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  JVal root;
  if (!JParser(text).parse(root) || root.kind != JVal::OBJ) {
    fprintf(stderr, "[tn] tuning table %s is not valid JSON; ignored\n", t.path.c_str());
    return t;
  }
  auto g = root.obj.find("gemm");
  if (g != root.obj.end() && g->second.kind == JVal::ARR)
    for (const JVal &r : g->second.arr) {
      if (r.kind != JVal::OBJ) continue;
      GemmRule q;
      q.bf16 = jstr(r, "prec") == "bf16x3";
      q.m3 = jstr(r, "form") == "3m";
      q.lm = jint(r, "lm", -1);
      q.ln = jint(r, "ln", -1);
      q.lk = jint(r, "lk", -1);
      q.tile = jint(r, "tile", 0);
      q.ksplit = jint(r, "ksplit", 0);
      if (q.lm >= 0 && q.ln >= 0 && q.lk >= 0) t.gemm.push_back(q);
    }
  auto tr = root.obj.find("tree");
  if (tr != root.obj.end() && tr->second.kind == JVal::ARR)
    for (const JVal &r : tr->second.arr) {
      if (r.kind != JVal::OBJ) continue;
      TreeRule q;
      q.fingerprint = strtoull(jstr(r, "fingerprint").c_str(), nullptr, 16);
      q.knobs.qw = jint(r, "qw", 0);
      q.knobs.spill = jint(r, "spill", (int)kTreeSpillElems);
      q.knobs.pack_nc = jint(r, "pack_nc", 64);
      if (q.fingerprint) t.tree.push_back(q);
    }
  t.loaded = true;
  return t;
}

const TuneTable &tune_table() {
  static const TuneTable t = load_table();
  return t;
}

static int ceil_log2(int64_t x) {
  int l = 0;
  while (((int64_t)1 << l) < x) ++l;
  return l;
}

const GemmRule *tune_gemm(bool bf16, bool m3, int64_t M, int64_t N, int64_t K) {
  const TuneTable &t = tune_table();
  const int lm = ceil_log2(M), ln = ceil_log2(N), lk = ceil_log2(K);
  for (const GemmRule &r : t.gemm)
    if (r.bf16 == bf16 && r.m3 == m3 && r.lm == lm && r.ln == ln && r.lk == lk) return &r;
  return nullptr;
}

const TreeKnobs *tune_tree(uint64_t fingerprint) {
  for (const TreeRule &r : tune_table().tree)
    if (r.fingerprint == fingerprint) return &r.knobs;
  return nullptr;
}

}  // namespace tn
