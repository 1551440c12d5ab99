// The tuning cache (xg_tune.cpp) under the sanitizers: a round trip through a
// file, then many damaged variants of a valid file (bytes flipped, cut,
// duplicated, deep nesting), each of which must either load or be refused
// whole, never crash, leak or read outside its buffers; and put/get from
// several threads at once.  Prints OK on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "xg.h"

namespace {

void fail(const char *what) {
  std::fprintf(stderr, "tune cache mismatch: %s\n", what);
  std::abort();
}

bool write_file(const std::string &path, const std::string &text) {
  std::FILE *f = std::fopen(path.c_str(), "wb");
  if (!f) return false;
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  return std::fclose(f) == 0 && ok;
}

std::string read_file(const std::string &path) {
  std::string out;
  std::FILE *f = std::fopen(path.c_str(), "rb");
  if (!f) return out;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) out.append(buf, n);
  std::fclose(f);
  return out;
}

}  // namespace

int main(int argc, char **argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  const std::string good_path = dir + "/good.json", bad_path = dir + "/bad.json";
  xg_tune_cache_clear();
  const xg_tune a{1, 1, 8, 1}, b{4, 8, 4, 4}, c{2, 2, 32, 0};
  if (xg_tune_cache_put("gfx950", 256, 0, "ragged/u32", &a, 7.25f) != XG_OK) fail("put a");
  if (xg_tune_cache_put("gfx950", 256, 1, "ragged/u32", &b, 1.5f) != XG_OK) fail("put b");
  if (xg_tune_cache_put("gfx942", 304, 2, "x y z", &c, NAN) != XG_OK) fail("put c");
  if (xg_tune_cache_save(good_path.c_str()) != XG_OK) fail("save");
  xg_tune_cache_clear();
  if (xg_tune_cache_load(good_path.c_str()) != XG_OK || xg_tune_cache_size() != 3) fail("round trip");
  xg_tune t;
  float ms;
  if (xg_tune_cache_get("gfx950", 256, 1, "ragged/u32", &t, &ms) != XG_OK || t.unroll != 8 || ms != 1.5f)
    fail("get b");
  const std::string good = read_file(good_path);
  std::mt19937_64 rng(12345);
  int loaded = 0, refused = 0;
  for (int it = 0; it < 3000; ++it) {
    std::string text = good;
    const int kind = (int)(rng() % 5);
    if (kind == 0) {                       // flip a few bytes
      for (int k = 0; k < 1 + (int)(rng() % 4); ++k) text[rng() % text.size()] = (char)(rng() & 0xFF);
    } else if (kind == 1) {                // cut anywhere
      text.resize(rng() % text.size());
    } else if (kind == 2) {                // duplicate a slice
      const size_t at = rng() % text.size(), len = rng() % 64;
      text.insert(at, text.substr(at, len));
    } else if (kind == 3) {                // deep nesting
      const int depth = (int)(rng() % 40);
      text = std::string(depth, '[') + text + std::string(depth, ']');
    } else {                               // a printable byte inserted
      text.insert(rng() % text.size(), 1, (char)(0x20 + rng() % 95));
    }
    if (!write_file(bad_path, text)) fail("write");
    xg_tune_cache_clear();
    const xg_status st = xg_tune_cache_load(bad_path.c_str());
    if (st == XG_OK) {
      ++loaded;
    } else if (st == XG_EINVAL) {
      if (xg_tune_cache_size() != 0) fail("a refused file merged entries");
      ++refused;
    } else {
      fail("unexpected status");
    }
  }
  if (refused < 1000) fail("too few damaged files refused");
  // put / get / size from several threads at once
  xg_tune_cache_clear();
  std::vector<std::thread> th;
  for (int k = 0; k < 8; ++k) {
    th.emplace_back([k] {
      char key[32];
      for (int i = 0; i < 200; ++i) {
        std::snprintf(key, sizeof key, "t%d/%d", k, i % 50);
        const xg_tune v{1u << (i % 5), 1u << (i % 4), 1 + (uint32_t)(i % 32), 1};
        if (xg_tune_cache_put("gfx950", 256, (uint32_t)(k % 3), key, &v, (float)i) != XG_OK) fail("thread put");
        xg_tune got;
        if (xg_tune_cache_get("gfx950", 256, (uint32_t)(k % 3), key, &got, nullptr) != XG_OK) fail("thread get");
        (void)xg_tune_cache_size();
      }
    });
  }
  for (auto &x : th) x.join();
  if (xg_tune_cache_size() != 8 * 50) fail("thread entries");
  std::printf("loaded %d refused %d\nOK\n", loaded, refused);
  return 0;
}
