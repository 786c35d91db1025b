// Host-side checks of libp3msr built with AddressSanitizer and
// UndefinedBehaviorSanitizer on its host code (tests/test_host_sanitizers.py
// builds and runs this on a machine without a GPU).  Every entry point is
// called along the paths that need no device: argument checks, error
// reporting, handle creation failing cleanly, and the autotuner cache
// parser on well-formed and malformed files.  Exit status 0 when every
// check holds; a sanitizer report aborts the run.
#include "p3msr.h"

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

static int failures = 0;

#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static bool err_has(const char *s) {
    const char *e = p3m_sr_last_error();
    return e && std::strstr(e, s) != nullptr;
}

static void write_file(const std::string &path, const std::string &text) {
    FILE *f = std::fopen(path.c_str(), "wb");
    if (!f) {
        std::fprintf(stderr, "cannot write %s\n", path.c_str());
        std::exit(2);
    }
    std::fwrite(text.data(), 1, text.size(), f);
    std::fclose(f);
}

static std::string entry(const char *device, long long n, int nt, int prec, int kind, int n_sub,
                         int ns, int target, int csize, int screen, int nsig) {
    char head[512];
    std::snprintf(head, sizeof(head),
                  "{\"device\": \"%s\", \"n\": %lld, \"nt\": %d, \"precision\": %d, "
                  "\"kind\": %d, \"n_sub\": %d, \"ns\": %d, \"target\": %d, \"csize\": %d, "
                  "\"screen\": %d, \"ms\": 1.5, \"sig\": [",
                  device, n, nt, prec, kind, n_sub, ns, target, csize, screen);
    std::string s = head;
    for (int k = 0; k < nsig; ++k) s += (k ? ", " : "") + std::to_string(k * 3);
    s += "]}";
    return s;
}

static void cache_checks(const std::string &dir) {
    int e = -1, l = -1;
    CHECK(p3m_sr_tune_cache_check(nullptr, &e, &l) == P3M_EINVAL);
    CHECK(p3m_sr_tune_cache_check((dir + "/missing.json").c_str(), &e, &l) == P3M_EINVAL);
    CHECK(err_has("cannot open"));

    const std::string good = entry("gfx950/x/256", 2097152, 45, 1, 0, 1, 1, 4096, 32, 2, 32);
    const std::string f1 = dir + "/good.json";
    write_file(f1, "[\n" + good + ",\n" + entry("d2", 10, 3, 0, 1, 8, 2, 1024, 16, 1, 32) + "\n]\n");
    CHECK(p3m_sr_tune_cache_check(f1.c_str(), &e, &l) == P3M_OK);
    CHECK(e == 2 && l == 4);
    CHECK(p3m_sr_tune_cache_check(f1.c_str(), nullptr, nullptr) == P3M_OK);

    // malformed entries are skipped, never read past their end
    std::string bad = "[\n";
    bad += good.substr(0, good.size() / 2) + "\n";                          // truncated
    bad += entry("d", 10, 3, 0, 0, 1, 1, 4096, 12, 1, 32) + "\n";          // bad csize
    bad += entry("d", 10, 3, 0, 0, 1, 1, 4096, 8, 2, 32) + "\n";           // screen 2, csize 8
    bad += entry("d", 10, 2, 0, 0, 1, 1, 4096, 32, 1, 32) + "\n";          // nt < 3
    bad += entry("d", -5, 3, 0, 0, 1, 1, 4096, 32, 1, 32) + "\n";          // n < 0
    bad += entry("d", 10, 3, 0, 0, 1, 99, 4096, 32, 1, 32) + "\n";         // ns > 16
    bad += entry("d", 10, 3, 0, 0, 1, 1, 4096, 32, 1, 20) + "\n";          // short signature
    bad += entry(std::string(400, 'x').c_str(), 10, 3, 0, 0, 1, 1, 4096, 32, 1, 32) + "\n";
    bad += "{\"device\": \"" + std::string(5000, 'y') + "\n";              // long, unterminated
    bad += std::string("{\"device\": \"a\", \"n\": 99999999999999999999999, \"nt\": 3}\n");
    bad += std::string("\x01\x02\xff{\"device\": \"\"\n", 17);
    bad += "{\"device\": \"z\", \"n\": 1e400, \"nt\": -2147483649}\n";
    bad += good + "\n";                                                     // one good line
    bad += "]";                                                             // no newline at end
    const std::string f2 = dir + "/bad.json";
    write_file(f2, bad);
    CHECK(p3m_sr_tune_cache_check(f2.c_str(), &e, &l) == P3M_OK);
    CHECK(e == 1);
    CHECK(l == 15);

    const std::string f3 = dir + "/empty.json";
    write_file(f3, "");
    CHECK(p3m_sr_tune_cache_check(f3.c_str(), &e, &l) == P3M_OK);
    CHECK(e == 0 && l == 0);

    // one line far longer than the reader's buffer, holding a good entry
    const std::string f4 = dir + "/long.json";
    write_file(f4, std::string(10000, ' ') + good + "\n");
    CHECK(p3m_sr_tune_cache_check(f4.c_str(), &e, &l) == P3M_OK);
    CHECK(e == 1 && l == 1);
}

static void argument_checks() {
    double *fake = reinterpret_cast<double *>(8);
    CHECK(p3m_sr_version() != nullptr && std::strncmp(p3m_sr_version(), "p3msr", 5) == 0);
    CHECK(p3m_sr_force(nullptr, fake, nullptr, nullptr, 10, 1.0, 0.01, 0.045, 1, fake, nullptr) ==
          P3M_EINVAL);
    CHECK(err_has("NULL handle"));
    CHECK(p3m_sr_force(nullptr, fake, nullptr, nullptr, -1, 1.0, 0.01, 0.045, 1, fake, nullptr) ==
          P3M_EINVAL);
    CHECK(p3m_sr_force(nullptr, fake, nullptr, nullptr, 10, 0.0, 0.01, 0.045, 1, fake, nullptr) ==
          P3M_EINVAL);
    CHECK(p3m_sr_force(nullptr, fake, nullptr, nullptr, 10, 1.0, 0.01, 0.6, 1, fake, nullptr) ==
          P3M_EINVAL);
    CHECK(p3m_sr_force(nullptr, fake, nullptr, nullptr, 10, 1.0, 0.01, 0.045, 7, fake, nullptr) ==
          P3M_EINVAL);
    CHECK(p3m_sr_force(nullptr, reinterpret_cast<double *>(12), nullptr, nullptr, 10, 1.0, 0.01,
                       0.045, 1, fake, nullptr) == P3M_EINVAL);
    CHECK(p3m_sr_force(nullptr, fake, nullptr, nullptr, (int64_t)1 << 31, 1.0, 0.01, 0.045, 1,
                       fake, nullptr) == P3M_EUNSUPPORTED);
    CHECK(p3m_sr_force_noalloc(nullptr, fake, nullptr, nullptr, (int64_t)1 << 20, 1.0, 0.01,
                               0.045, 1, fake, nullptr) != P3M_OK);
    CHECK(p3m_sr_force_backward(nullptr, fake, nullptr, nullptr, 10, 1.0, 0.01, 0.045, 1,
                                nullptr, fake, nullptr) == P3M_EINVAL);
    const uint8_t thr[2] = {0, 3};
    CHECK(p3m_sr_force_batched(nullptr, fake, nullptr, reinterpret_cast<uint8_t *>(8), 10, 0, thr,
                               1.0, 0.01, 0.045, 1, fake, nullptr) == P3M_EINVAL);
    CHECK(p3m_sr_force_batched(nullptr, fake, nullptr, reinterpret_cast<uint8_t *>(8), 10, 2,
                               nullptr, 1.0, 0.01, 0.045, 1, fake, nullptr) == P3M_EINVAL);
    CHECK(p3m_sr_set_config(nullptr, 17, 0, 0, -1) == P3M_EINVAL);
    CHECK(p3m_sr_set_config(nullptr, 2, 0, 12, -1) == P3M_EINVAL);
    CHECK(p3m_sr_set_shape(nullptr, 5, 0) == P3M_EINVAL);
    CHECK(p3m_sr_set_softening(nullptr, -1.0) == P3M_EINVAL);
    CHECK(p3m_sr_set_deterministic(nullptr, 2) == P3M_EINVAL);
    CHECK(p3m_sr_set_debug_limits(nullptr, -1, -1) == P3M_EINVAL);
    CHECK(p3m_sr_set_debug_limits(nullptr, 0, -3) == P3M_EINVAL);
    CHECK(p3m_sr_set_timing(nullptr, 1) == P3M_EINVAL);
    CHECK(p3m_sr_set_tune_cache(nullptr, "x") == P3M_EINVAL);
    CHECK(p3m_sr_tune_status(nullptr, nullptr, nullptr) == P3M_EINVAL);
    p3m_sr_stats st;
    CHECK(p3m_sr_get_stats(nullptr, &st) == P3M_EINVAL);
    CHECK(p3m_sr_autotune(nullptr, fake, nullptr, nullptr, 10, 1.0, 0.01, 0.045, 1, 9, fake,
                          nullptr) == P3M_EINVAL);
    CHECK(p3m_lr_force(nullptr, fake, nullptr, nullptr, 10, 1.0, 48, 0.02, fake, nullptr) ==
          P3M_EINVAL);
    CHECK(p3m_sr_destroy(nullptr) == P3M_OK || p3m_sr_destroy(nullptr) == P3M_EINVAL);
    // a long message is cut to the error buffer, not written past it
    std::string longpath(3000, 'p');
    CHECK(p3m_sr_tune_cache_check(longpath.c_str(), nullptr, nullptr) == P3M_EINVAL);
    CHECK(std::strlen(p3m_sr_last_error()) < 1024);
}

static void create_without_gpu() {
    p3m_sr_handle h = nullptr;
    const int rc = p3m_sr_create(&h, 0);
    if (rc == P3M_OK) {
        // a GPU is visible after all: the handle must still close cleanly
        CHECK(h != nullptr);
        CHECK(p3m_sr_destroy(h) == P3M_OK);
    } else {
        CHECK(h == nullptr);
        CHECK(std::strlen(p3m_sr_last_error()) > 0);
    }
    CHECK(p3m_sr_create(nullptr, 0) == P3M_EINVAL);
    CHECK(p3m_sr_create(&h, -1) != P3M_OK);
}

int main(int argc, char **argv) {
    if (argc < 2) {
        std::fprintf(stderr, "usage: host_checks <scratch dir>\n");
        return 2;
    }
    argument_checks();
    cache_checks(argv[1]);
    create_without_gpu();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
