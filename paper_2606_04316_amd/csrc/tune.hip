// tune.hip -- launch choices of a plan and the tuning cache (host code).
//
// The choices (integral schedule, first-half workgroup order, second-quarter
// GEMM tile) are picked per plan by qdcb_plan_autotune (transform.hip) and
// remembered across processes in a text file of JSON lines keyed by the
// plan's shape.
#include <cstdlib>

#include "plan.h"

using namespace qdcb;

namespace qdcb {

const char *tune_problem(const qdcb_plan &p, const qdcb_tune &t) {
  if (t.eri_sched != 0 && t.eri_sched != 1) return "eri_sched must be 0 or 1";
  if (t.fh_order != 0 && t.fh_order != 1) return "fh_order must be 0 or 1";
  if (t.sq_tile != 64 && t.sq_tile != 128) return "sq_tile must be 64 or 128";
  if (t.sq_tile == 128 && p.n % 2) return "sq_tile 128 needs an even n_mo";
  if (t.reserved != 0) return "reserved must be 0";
  return nullptr;
}

}  // namespace qdcb

namespace {

bool key_ok(const char *k) {
  for (; *k; ++k)
    if (*k == '"' || *k == '\n' || *k == '\r' || *k == '\\') return false;
  return true;
}

// value of "name": <int> in a line, or false
bool field(const char *line, const char *name, int *v) {
  std::string pat = std::string("\"") + name + "\":";
  const char *f = std::strstr(line, pat.c_str());
  return f && std::sscanf(f + pat.size(), " %d", v) == 1;
}

}  // namespace

extern "C" {

qdcb_status qdcb_plan_set_tune(qdcb_plan *p, const qdcb_tune *t) {
  return guarded([&] {
    if (!p || !t) fail(QDCB_E_INVALID, "NULL argument");
    PlanUse use(*p);
    if (const char *why = tune_problem(*p, *t)) fail(QDCB_E_INVALID, why);
    p->tune = *t;
  });
}

qdcb_status qdcb_plan_get_tune(const qdcb_plan *p, qdcb_tune *t) {
  return guarded([&] {
    if (!p || !t) fail(QDCB_E_INVALID, "NULL argument");
    *t = p->tune;
  });
}

qdcb_status qdcb_plan_set_mo_batch(qdcb_plan *p, int32_t pairs) {
  return guarded([&] {
    if (!p) fail(QDCB_E_INVALID, "NULL argument");
    PlanUse use(*p);
    if (pairs < 0) fail(QDCB_E_INVALID, "pairs must be >= 0");
    if (pairs > 0 && p->spinor) fail(QDCB_E_UNSUPPORTED, "the MO-driven variant is for quaternion plans");
    p->mo_batch = pairs;
  });
}

qdcb_status qdcb_plan_tune_key(const qdcb_plan *p, char *buf, size_t len) {
  return guarded([&] {
    if (!p || !buf) fail(QDCB_E_INVALID, "NULL argument");
    if (len < p->tune_key.size() + 1) fail(QDCB_E_INVALID, "key buffer too small");
    std::memcpy(buf, p->tune_key.c_str(), p->tune_key.size() + 1);
  });
}

qdcb_status qdcb_tune_cache_lookup(const char *path, const char *key, qdcb_tune *t,
                                   int32_t *found) {
  return guarded([&] {
    if (!path || !key || !t || !found) fail(QDCB_E_INVALID, "NULL argument");
    *found = 0;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    std::string want = std::string("\"key\": \"") + key + "\"";
    std::vector<char> line(4096);
    while (std::fgets(line.data(), (int)line.size(), f)) {
      if (!std::strstr(line.data(), want.c_str())) continue;
      qdcb_tune c{};
      if (field(line.data(), "eri_sched", &c.eri_sched) &&
          field(line.data(), "fh_order", &c.fh_order) &&
          field(line.data(), "sq_tile", &c.sq_tile) && (c.eri_sched == 0 || c.eri_sched == 1) &&
          (c.fh_order == 0 || c.fh_order == 1) && (c.sq_tile == 64 || c.sq_tile == 128)) {
        *t = c;
        *found = 1;
      }
    }
    std::fclose(f);
  });
}

qdcb_status qdcb_tune_cache_store(const char *path, const char *key, const qdcb_tune *t) {
  return guarded([&] {
    if (!path || !key || !t) fail(QDCB_E_INVALID, "NULL argument");
    if (!key_ok(key)) fail(QDCB_E_INVALID, "key holds a quote, backslash or line break");
    FILE *f = std::fopen(path, "a");
    if (!f) fail(QDCB_E_INVALID, std::string("cannot open tuning cache ") + path);
    std::fprintf(f, "{\"key\": \"%s\", \"eri_sched\": %d, \"fh_order\": %d, \"sq_tile\": %d}\n",
                 key, t->eri_sched, t->fh_order, t->sq_tile);
    std::fclose(f);
  });
}

}  // extern "C"
