// Checkpoint header of a surrogate network (host code only): the magic line
// and the one-line JSON header that hsd_surrogate_save writes, parsed and
// checked before any payload byte is used.  Shared by the library and the
// sanitizer test harness, which feeds it truncated and corrupted images.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <string>

namespace hsd {

struct CkptHeader {
    long long n_params = 0;
    long long step = 0;        // Adam steps taken (also the minibatch generator's position)
    bool optimizer = false;    // the Adam moments follow the statistics
    double band_weight = 0.0;  // the loss setting
    size_t payload_off = 0;    // first byte after the header line
};

// The number after "key": in a one-line JSON header, or false.
inline bool ckpt_json_integer(const std::string& h, const char* key, long long& out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = h.find(k);
    if (at == std::string::npos) return false;
    const char* p = h.c_str() + at + k.size();
    char* end = nullptr;
    out = std::strtoll(p, &end, 10);
    return end != p;
}

inline bool ckpt_json_real(const std::string& h, const char* key, double& out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = h.find(k);
    if (at == std::string::npos) return false;
    const char* p = h.c_str() + at + k.size();
    char* end = nullptr;
    out = std::strtod(p, &end);
    return end != p;
}

inline bool ckpt_json_bool(const std::string& h, const char* key, bool& out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = h.find(k);
    if (at == std::string::npos) return false;
    size_t q = at + k.size();
    while (q < h.size() && h[q] == ' ') ++q;
    if (h.compare(q, 4, "true") == 0) out = true;
    else if (h.compare(q, 5, "false") == 0) out = false;
    else return false;
    return true;
}

// Payload bytes of a network with n_params parameters and n_out outputs:
// params, x_mean [33], x_std [33], y_mean [n_out], y_std [n_out], and the two
// Adam moments when present (FP32 each).
inline size_t ckpt_payload_bytes(long long n_params, int n_out, bool optimizer) {
    const long long floats = n_params * (optimizer ? 3 : 1) + 2LL * 33 + 2LL * n_out;
    return sizeof(float) * static_cast<size_t>(floats);
}

// Checks the image `data` of a checkpoint file against a network of the
// given widths (the last one the output count) and parameter count, down to
// its exact size; "" and the header in `out` when it fits, else the reason.
inline std::string ckpt_parse(const std::string& data, const int (&widths)[5], long long n_params, CkptHeader& out) {
    const std::string magic = "HSDSUR 1\n";
    if (data.compare(0, magic.size(), magic) != 0) return "not a surrogate checkpoint";
    const size_t eol = data.find('\n', magic.size());
    if (eol == std::string::npos) return "truncated header";
    const std::string h = data.substr(magic.size(), eol - magic.size());
    CkptHeader c;
    if (!ckpt_json_integer(h, "n_params", c.n_params) || !ckpt_json_integer(h, "step", c.step) ||
        !ckpt_json_bool(h, "optimizer", c.optimizer) || !ckpt_json_real(h, "loss_band_weight", c.band_weight) ||
        h.find("\"byte_order\": \"little\"") == std::string::npos)
        return "malformed header";
    if (!(c.band_weight >= 0.0 && c.band_weight <= 1.0)) return "loss_band_weight outside [0, 1]";
    std::string want = "\"widths\": [";
    for (int i = 0; i < 5; ++i) want += std::to_string(widths[i]) + (i < 4 ? ", " : "]");
    if (h.find(want) == std::string::npos || c.n_params != n_params) return "checkpoint of a network of another shape";
    if (c.step < 0) return "negative step count";
    c.payload_off = eol + 1;
    if (data.size() != c.payload_off + ckpt_payload_bytes(n_params, widths[4], c.optimizer))
        return "checkpoint size does not match its header";
    out = c;
    return "";
}

}  // namespace hsd
