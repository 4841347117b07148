// Host-side sanitizer harness for the checkpoint header parser (built with
// g++ -fsanitize=address,undefined by tests/test_host_sanitize.py; no GPU
// code).  A valid image is built the way hsd_surrogate_save lays it out, then
// every truncation, seeded byte corruptions and edited headers are parsed:
// the parser must accept the valid image, reject every truncation and every
// header that no longer matches, and never read out of bounds.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "hsd_ckpt.h"

namespace {

std::string header(const int (&w)[5], long long np, long long step, const char* opt, const char* bw,
                   const char* order) {
    std::string h = "{\"format\": \"hsd-surrogate\", \"widths\": [";
    for (int i = 0; i < 5; ++i) h += std::to_string(w[i]) + (i < 4 ? ", " : "]");
    h += ", \"n_params\": " + std::to_string(np) + ", \"step\": " + std::to_string(step) +
         ", \"loss_band_weight\": " + bw + ", \"optimizer\": " + opt + ", \"byte_order\": \"" + order + "\"}";
    return h;
}

std::string image(const std::string& h, size_t payload) {
    std::string d = "HSDSUR 1\n" + h + "\n";
    d.append(payload, '\x01');
    return d;
}

int fails = 0;

void expect(bool ok, const char* what, size_t detail = 0) {
    if (!ok) {
        std::printf("FAIL: %s (%zu)\n", what, detail);
        ++fails;
    }
}

}  // namespace

int main() {
    // a small network keeps the all-truncations sweep fast; the parser reads
    // only the header, whose layout does not depend on the widths
    const int w[5] = {33, 8, 8, 8, 5};
    const long long np = 33LL * 8 + 8 + 2 * (8LL * 8 + 8) + 8LL * 5 + 5;
    hsd::CkptHeader out;
    for (const bool opt : {true, false}) {
        const size_t payload = hsd::ckpt_payload_bytes(np, w[4], opt);
        const std::string good = image(header(w, np, 1234, opt ? "true" : "false", "0.25", "little"), payload);
        expect(hsd::ckpt_parse(good, w, np, out).empty(), "valid image rejected");
        expect(out.step == 1234 && out.optimizer == opt && out.band_weight == 0.25 && out.n_params == np,
               "valid header misread");
        // every truncation is rejected
        for (size_t n = 0; n < good.size(); ++n) {
            const std::string cut = good.substr(0, n);
            expect(!hsd::ckpt_parse(cut, w, np, out).empty(), "truncation accepted", n);
        }
        // seeded corruptions of the header bytes: any verdict, but no memory error
        unsigned long long x = 4627;
        const size_t hdr_end = good.find('\n', 9) + 1;
        for (int it = 0; it < 20000; ++it) {
            std::string bad = good;
            for (int k = 0; k < 3; ++k) {
                x = x * 6364136223846793005ULL + 1442695040888963407ULL;
                const size_t at = static_cast<size_t>(x >> 33) % hdr_end;
                bad[at] = static_cast<char>(x >> 17);
            }
            (void)hsd::ckpt_parse(bad, w, np, out);
            // the same corruption with the image cut right after the header
            (void)hsd::ckpt_parse(bad.substr(0, hdr_end), w, np, out);
        }
        // edited headers
        expect(!hsd::ckpt_parse(image(header(w, np + 1, 0, "true", "0", "little"), payload), w, np, out).empty(),
               "wrong n_params accepted");
        expect(!hsd::ckpt_parse(image(header(w, np, -1, "true", "0", "little"), payload), w, np, out).empty(),
               "negative step accepted");
        expect(!hsd::ckpt_parse(image(header(w, np, 0, "maybe", "0", "little"), payload), w, np, out).empty(),
               "bad boolean accepted");
        expect(!hsd::ckpt_parse(image(header(w, np, 0, "true", "1.5", "little"), payload), w, np, out).empty(),
               "band weight above 1 accepted");
        expect(!hsd::ckpt_parse(image(header(w, np, 0, "true", "nan", "little"), payload), w, np, out).empty(),
               "NaN band weight accepted");
        expect(!hsd::ckpt_parse(image(header(w, np, 0, "true", "0", "big"), payload), w, np, out).empty(),
               "big-endian image accepted");
        const int w2[5] = {33, 8, 8, 8, 6};
        expect(!hsd::ckpt_parse(good, w2, np, out).empty(), "other output width accepted");
        expect(!hsd::ckpt_parse(image(header(w, np, 0, opt ? "false" : "true", "0", "little"), payload), w, np, out)
                    .empty(),
               "optimizer flag that does not match the size accepted");
        expect(!hsd::ckpt_parse(good + "x", w, np, out).empty(), "trailing byte accepted");
        expect(!hsd::ckpt_parse("HSDSUR 1\n{\"n_params\": 99999999999999999999999}\n", w, np, out).empty(),
               "overflowing header accepted");
    }
    std::printf("%s: %d failures\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
