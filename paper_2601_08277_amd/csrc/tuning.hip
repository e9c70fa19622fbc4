// Density-based path choice of PIC_PATH_AUTO. The paper runs the matrix kernel where cells
// are dense and falls back to vector kernels where they are sparse (Sec. 6.1, LWFA; Sec. 7);
// on gfx950 the break-even density is measured, not assumed: the autotuner times every path
// that meets the float32 tolerance per (shape order, particles-per-cell bucket) and writes
// the fastest as "path" into its JSON cache, which pic_tuning_load reads. Without a loaded
// cache AUTO takes the per-cell VALU path (the fastest at every density measured).
#include <cmath>
#include <fstream>
#include <mutex>
#include <sstream>
#include <vector>

#include "pic_host.h"

namespace {
struct AutoRule {
  int order;
  double ppc;
  int path;
};
std::mutex g_rules_mu;
std::vector<AutoRule> g_rules;

int path_of_name(const std::string& s) {
  if (s == "cell_valu") return PIC_PATH_CELL_VALU;
  if (s == "mfma_fp16") return PIC_PATH_MFMA_FP16;
  if (s == "mfma_bf16") return PIC_PATH_MFMA_BF16;
  if (s == "atomic") return PIC_PATH_ATOMIC;
  return -1;
}

// Value after "key": inside [b, e): a number, or a quoted string (quotes stripped).
bool field(const std::string& t, size_t b, size_t e, const char* key, std::string& out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = t.find(k, b);
  if (p == std::string::npos || p >= e) return false;
  p = t.find(':', p + k.size());
  if (p == std::string::npos || p >= e) return false;
  ++p;
  while (p < e && (t[p] == ' ' || t[p] == '\n' || t[p] == '\t' || t[p] == '\r')) ++p;
  if (p >= e) return false;
  if (t[p] == '"') {
    const size_t q = t.find('"', p + 1);
    if (q == std::string::npos || q >= e) return false;
    out = t.substr(p + 1, q - p - 1);
    return true;
  }
  size_t q = p;
  while (q < e && t[q] != ',' && t[q] != '}' && t[q] != '\n') ++q;
  out = t.substr(p, q - p);
  return true;
}
}  // namespace

extern "C" pic_status pic_tuning_load(const char* json_path) {
  std::vector<AutoRule> rules;
  if (json_path) {
    std::ifstream f(json_path);
    if (!f) return set_error(PIC_ERR_INVALID_ARG, std::string("cannot read ") + json_path);
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t p = t.find("\"entries\"");
    if (p == std::string::npos) return set_error(PIC_ERR_INVALID_ARG, "no \"entries\" list");
    p = t.find('[', p);
    if (p == std::string::npos) return set_error(PIC_ERR_INVALID_ARG, "malformed \"entries\"");
    // walk the list; each entry's own fields are read with its nested objects and lists
    // blanked out (so keys inside "ms_paths" or "tile" are not mistaken for its own)
    int depth = 0;
    size_t ent = std::string::npos;
    std::string top;
    for (size_t i = p; i < t.size(); ++i) {
      const char ch = t[i];
      if (ch == '"') {                       // skip strings
        const size_t q = t.find('"', i + 1);
        if (q == std::string::npos) break;
        if (depth == 2) top.append(t, i, q - i + 1);
        i = q;
        continue;
      }
      if (ch == '[' || ch == '{') {
        ++depth;
        if (depth == 2 && ch == '{') {
          ent = i;
          top = "{";
        } else if (depth > 2) {
          top.push_back(' ');
        }
        continue;
      }
      if (ch == ']' || ch == '}') {
        --depth;
        if (depth == 1 && ch == '}' && ent != std::string::npos) {
          top.push_back('}');
          std::string so, sp, sn;
          if (!field(top, 0, top.size(), "order", so) || !field(top, 0, top.size(), "ppc", sp) ||
              !field(top, 0, top.size(), "path", sn))
            return set_error(PIC_ERR_INVALID_ARG, "entry without order, ppc or path");
          AutoRule r{std::atoi(so.c_str()), std::atof(sp.c_str()), path_of_name(sn)};
          if (r.order < 1 || r.order > 3 || !(r.ppc > 0.0) || r.path < 0)
            return set_error(PIC_ERR_INVALID_ARG, "entry with a bad order, ppc or path name");
          rules.push_back(r);
          ent = std::string::npos;
        }
        if (depth == 0) break;               // end of the entries list
        continue;
      }
      if (depth == 2) top.push_back(ch);
    }
    if (depth != 0) return set_error(PIC_ERR_INVALID_ARG, "unterminated \"entries\" list");
  }
  std::lock_guard<std::mutex> lk(g_rules_mu);
  g_rules.swap(rules);
  return PIC_OK;
}

// Particles per cell of the bins: the count of the newest rebin statistics the host holds,
// else the slot count the caller sized for its slack.
static double bins_density(const pic_bins* b) {
  for (auto it = b->history.rbegin(); it != b->history.rend(); ++it)
    if (it->complete && it->n_valid > 0) return (double)it->n_valid / (double)b->kb.nbins;
  return (double)b->nslots / ((1.0 + b->slack) * (double)b->kb.nbins);
}

int choose_path(const KGrid& G, const pic_bins* b) {
  if (!b || b->kb.nbins <= 0) return PIC_PATH_CELL_VALU;
  const double ppc = std::max(bins_density(b), 1e-3);
  std::lock_guard<std::mutex> lk(g_rules_mu);
  int best = PIC_PATH_CELL_VALU;
  double bd = 0.0;
  bool any = false;
  for (const AutoRule& r : g_rules) {
    if (r.order != G.order) continue;
    const double d = std::fabs(std::log(ppc) - std::log(r.ppc));
    if (!any || d < bd) {
      any = true;
      bd = d;
      best = r.path;
    }
  }
  return best;
}

extern "C" int pic_auto_path(const pic_grid* grid, const pic_bins* bins) {
  if (validate_grid(grid) != PIC_OK || !bins) return PIC_PATH_CELL_VALU;
  return choose_path(make_kgrid(*grid), bins);
}
