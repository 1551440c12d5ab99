// Tuning cache of libxg (include/xg.h): batch launch shapes keyed by (device
// architecture, compute units, family member, workload key), held per process
// and stored as JSON.  Host-only (no HIP headers), so the sanitizer tests can
// build it with a plain host compiler.
#include <cctype>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "xg.h"

namespace {

constexpr size_t kMaxKey = 256;  // longest arch or workload key accepted

struct Key {
  std::string arch;
  uint32_t cus;
  uint32_t family;
  std::string key;
  bool operator<(const Key &o) const {
    return std::tie(arch, cus, family, key) < std::tie(o.arch, o.cus, o.family, o.key);
  }
};

struct Entry {
  xg_tune tune;
  double ms;
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;
std::once_flag g_env_once;

bool name_ok(const char *s) {
  if (!s) return false;
  const size_t n = std::strlen(s);
  if (n == 0 || n > kMaxKey) return false;
  for (size_t i = 0; i < n; ++i)
    if ((unsigned char)s[i] < 0x20 || s[i] == '"' || s[i] == '\\') return false;
  return true;
}

// The launch shapes the batch kernels accept (as xg_generate_batch_planned
// checks them; store_words 0 means the default for the unroll).
bool tune_ok(const xg_tune &t) {
  const uint32_t w = t.waves_per_block, u = t.unroll;
  const bool wpb = w == 1 || w == 2 || w == 4 || w == 8 || w == 16;
  const bool un = u == 1 || u == 2 || u == 4 || u == 8;
  const bool sw = t.store_words == 0 || t.store_words == 1 || (t.store_words == 4 && u >= 4);
  return wpb && un && sw && t.blocks_per_cu >= 1 && t.blocks_per_cu <= 32;
}

// ---- a small JSON reader for the cache file ----------------------------------
// Values: objects, arrays, strings, numbers, true / false / null.

struct JValue {
  enum Type { kNull, kBool, kNum, kStr, kArr, kObj } type = kNull;
  double num = 0;
  bool b = false;
  std::string str;
  std::vector<JValue> arr;
  std::vector<std::pair<std::string, JValue>> obj;
  const JValue *get(const char *name) const {
    for (const auto &kv : obj)
      if (kv.first == name) return &kv.second;
    return nullptr;
  }
};

struct Reader {
  const char *p, *end;
  int depth = 0;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool lit(const char *w) {
    const size_t n = std::strlen(w);
    if ((size_t)(end - p) < n || std::strncmp(p, w, n) != 0) return false;
    p += n;
    return true;
  }
  bool string(std::string &out) {
    if (p >= end || *p != '"') return false;
    ++p;
    while (p < end && *p != '"') {
      char c = *p++;
      if ((unsigned char)c < 0x20) return false;
      if (c == '\\') {
        if (p >= end) return false;
        const char e = *p++;
        switch (e) {
          case '"': c = '"'; break;
          case '\\': c = '\\'; break;
          case '/': c = '/'; break;
          case 'b': c = '\b'; break;
          case 'f': c = '\f'; break;
          case 'n': c = '\n'; break;
          case 'r': c = '\r'; break;
          case 't': c = '\t'; break;
          case 'u': {  // ASCII code points only
            if (end - p < 4) return false;
            unsigned v = 0;
            for (int i = 0; i < 4; ++i) {
              const char h = p[i];
              v = v * 16 + (h >= '0' && h <= '9' ? h - '0' : h >= 'a' && h <= 'f' ? h - 'a' + 10
                                                            : h >= 'A' && h <= 'F' ? h - 'A' + 10 : 99);
              if (v > 0xFFFF) return false;
            }
            if (v == 0 || v > 0x7F) return false;
            p += 4;
            c = (char)v;
            break;
          }
          default: return false;
        }
      }
      out.push_back(c);
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool number(double &out) {
    const char *s = p;
    if (p < end && *p == '-') ++p;
    while (p < end && (std::isdigit((unsigned char)*p) || *p == '.' || *p == 'e' || *p == 'E' || *p == '+' ||
                       *p == '-'))
      ++p;
    if (p == s) return false;
    const std::string t(s, p);
    char *stop = nullptr;
    errno = 0;
    out = std::strtod(t.c_str(), &stop);
    return stop == t.c_str() + t.size() && errno == 0 && std::isfinite(out);
  }
  bool value(JValue &v) {
    if (++depth > 16) return false;
    ws();
    bool ok = false;
    if (p >= end) {
      ok = false;
    } else if (*p == '{') {
      ++p;
      v.type = JValue::kObj;
      ws();
      if (p < end && *p == '}') {
        ++p;
        ok = true;
      } else {
        for (;;) {
          ws();
          std::string name;
          JValue item;
          if (!string(name)) break;
          ws();
          if (p >= end || *p != ':') break;
          ++p;
          if (!value(item)) break;
          v.obj.emplace_back(std::move(name), std::move(item));
          ws();
          if (p < end && *p == ',') {
            ++p;
            continue;
          }
          if (p < end && *p == '}') {
            ++p;
            ok = true;
          }
          break;
        }
      }
    } else if (*p == '[') {
      ++p;
      v.type = JValue::kArr;
      ws();
      if (p < end && *p == ']') {
        ++p;
        ok = true;
      } else {
        for (;;) {
          JValue item;
          if (!value(item)) break;
          v.arr.push_back(std::move(item));
          ws();
          if (p < end && *p == ',') {
            ++p;
            continue;
          }
          if (p < end && *p == ']') {
            ++p;
            ok = true;
          }
          break;
        }
      }
    } else if (*p == '"') {
      v.type = JValue::kStr;
      ok = string(v.str);
    } else if (lit("true")) {
      v.type = JValue::kBool;
      v.b = true;
      ok = true;
    } else if (lit("false")) {
      v.type = JValue::kBool;
      ok = true;
    } else if (lit("null")) {
      ok = true;
    } else {
      v.type = JValue::kNum;
      ok = number(v.num);
    }
    --depth;
    return ok;
  }
};

bool as_u32(const JValue *v, uint32_t *out) {
  if (!v || v->type != JValue::kNum || v->num < 0 || v->num > 4294967295.0 || v->num != std::floor(v->num))
    return false;
  *out = (uint32_t)v->num;
  return true;
}

// Parses a cache file's text into entries; false if it is not one.
bool parse_cache(const std::string &text, std::vector<std::pair<Key, Entry>> *out) {
  Reader r{text.data(), text.data() + text.size()};
  JValue root;
  if (!r.value(root)) return false;
  r.ws();
  if (r.p != r.end || root.type != JValue::kObj) return false;
  const JValue *ver = root.get("xg_tune_cache");
  uint32_t version = 0;
  if (!as_u32(ver, &version) || version != 1) return false;
  const JValue *entries = root.get("entries");
  if (!entries || entries->type != JValue::kArr) return false;
  for (const JValue &e : entries->arr) {
    if (e.type != JValue::kObj) return false;
    const JValue *arch = e.get("arch"), *key = e.get("key"), *ms = e.get("ms");
    Key k;
    Entry en{};
    if (!arch || arch->type != JValue::kStr || !key || key->type != JValue::kStr) return false;
    k.arch = arch->str;
    k.key = key->str;
    if (!name_ok(k.arch.c_str()) || !name_ok(k.key.c_str()) || k.arch.size() != std::strlen(k.arch.c_str()) ||
        k.key.size() != std::strlen(k.key.c_str()))
      return false;
    if (!as_u32(e.get("cus"), &k.cus) || !as_u32(e.get("family"), &k.family) ||
        !as_u32(e.get("waves_per_block"), &en.tune.waves_per_block) || !as_u32(e.get("unroll"), &en.tune.unroll) ||
        !as_u32(e.get("blocks_per_cu"), &en.tune.blocks_per_cu) ||
        !as_u32(e.get("store_words"), &en.tune.store_words))
      return false;
    if (k.family > XG_FAMILY_R64_W64 || !tune_ok(en.tune)) return false;
    en.ms = -1.0;
    if (ms) {
      if (ms->type != JValue::kNum) return false;
      en.ms = ms->num;
    }
    out->emplace_back(std::move(k), en);
  }
  return true;
}

xg_status load_locked(const char *path) {
  std::FILE *f = std::fopen(path, "rb");
  if (!f) return XG_EINVAL;
  std::string text;
  char buf[4096];
  size_t got;
  bool too_big = false;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) {
    text.append(buf, got);
    if (text.size() > (64u << 20)) {
      too_big = true;
      break;
    }
  }
  const bool read_error = std::ferror(f) != 0;
  std::fclose(f);
  if (too_big || read_error) return XG_EINVAL;
  std::vector<std::pair<Key, Entry>> entries;
  if (!parse_cache(text, &entries)) return XG_EINVAL;
  for (auto &kv : entries) g_cache[kv.first] = kv.second;
  return XG_OK;
}

// The cache named by XG_TUNE_CACHE is merged in once, before the first
// lookup (a missing or malformed file is ignored).
void load_env_once() {
  std::call_once(g_env_once, [] {
    const char *path = std::getenv("XG_TUNE_CACHE");
    if (!path || !*path) return;
    try {
      std::lock_guard<std::mutex> lock(g_mu);
      (void)load_locked(path);
    } catch (const std::bad_alloc &) {
    }
  });
}

}  // namespace

extern "C" {

xg_status xg_tune_cache_load(const char *path) {
  if (!path) return XG_EINVAL;
  try {
    std::lock_guard<std::mutex> lock(g_mu);
    return load_locked(path);
  } catch (const std::bad_alloc &) {
    return XG_ENOMEM;
  }
}

xg_status xg_tune_cache_save(const char *path) {
  if (!path) return XG_EINVAL;
  try {
    std::string text = "{\"xg_tune_cache\": 1, \"entries\": [";
    {
      std::lock_guard<std::mutex> lock(g_mu);
      bool first = true;
      for (const auto &kv : g_cache) {
        char num[512];
        std::snprintf(num, sizeof num,
                      "\"cus\": %u, \"family\": %u, \"waves_per_block\": %u, \"unroll\": %u, "
                      "\"blocks_per_cu\": %u, \"store_words\": %u, \"ms\": %.6g}",
                      kv.first.cus, kv.first.family, kv.second.tune.waves_per_block, kv.second.tune.unroll,
                      kv.second.tune.blocks_per_cu, kv.second.tune.store_words, kv.second.ms);
        text += first ? "\n  {" : ",\n  {";
        text += "\"arch\": \"" + kv.first.arch + "\", \"key\": \"" + kv.first.key + "\", ";
        text += num;
        first = false;
      }
    }
    text += "\n]}\n";
    const std::string tmp = std::string(path) + ".tmp";
    std::FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return XG_EINVAL;
    const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
    if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path) != 0) {
      std::remove(tmp.c_str());
      return XG_EINVAL;
    }
    return XG_OK;
  } catch (const std::bad_alloc &) {
    return XG_ENOMEM;
  }
}

xg_status xg_tune_cache_put(const char *arch, uint32_t cus, uint32_t family, const char *tune_key,
                            const xg_tune *tune, float ms) {
  if (!name_ok(arch) || !name_ok(tune_key) || !tune || cus == 0 || family > XG_FAMILY_R64_W64 || !tune_ok(*tune))
    return XG_EINVAL;
  load_env_once();
  try {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache[Key{arch, cus, family, tune_key}] = Entry{*tune, std::isfinite(ms) ? (double)ms : -1.0};
  } catch (const std::bad_alloc &) {
    return XG_ENOMEM;
  }
  return XG_OK;
}

xg_status xg_tune_cache_get(const char *arch, uint32_t cus, uint32_t family, const char *tune_key, xg_tune *tune,
                            float *ms) {
  if (!name_ok(arch) || !name_ok(tune_key) || !tune) return XG_EINVAL;
  load_env_once();
  try {
    std::lock_guard<std::mutex> lock(g_mu);
    const auto it = g_cache.find(Key{arch, cus, family, tune_key});
    if (it == g_cache.end()) return XG_ERANGE;
    *tune = it->second.tune;
    if (ms) *ms = (float)it->second.ms;
  } catch (const std::bad_alloc &) {
    return XG_ENOMEM;
  }
  return XG_OK;
}

uint32_t xg_tune_cache_size(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  return (uint32_t)g_cache.size();
}

void xg_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_cache.clear();
}

}  // extern "C"
