// The model file's header parser (paper_2304_09409_amd/csrc/json_header.h) on input it does not
// control: a valid header as the library writes it, every truncation of it, random byte
// mutations of it, and nesting past the depth limit. Built with the host sanitizers by
// tests/test_oracle_sanitize.py: any read past the buffer or undefined operation fails the run;
// the valid header must parse, the truncated ones must be refused.
#include <cstdio>
#include <random>
#include <string>

#include "json_header.h"

using dpk::json::JParser;
using dpk::json::JVal;

static bool parse(const std::string& s, JVal* out = nullptr)
{
    JParser jp{s.data(), s.data() + s.size()};
    JVal v = jp.value(0);
    if (out) *out = v;
    return jp.ok && v.kind == JVal::OBJ;
}

int main()
{
    const std::string good =
        "{\"format\": \"dpk-se_e2_a\", \"version\": 1, \"ntypes\": 2, \"sel\": [46, 92], \"rcut\": 6.0, "
        "\"rcut_smth\": 0.5, \"embedding\": [25, 50, 100], \"axis\": 16, \"fitting\": [240, 240, 240], "
        "\"type_one_side\": false, \"descriptor\": \"se_e2_a\", \"nparams\": 1234, "
        "\"compression\": {\"stride\": 0.01, \"x_max\": 2.7}, \"note\": \"a \\\"quoted\\\" string\\n\"}";
    JVal root;
    if (!parse(good, &root)) { std::printf("valid header refused\n"); return 1; }
    int32_t nt = 0, sel[2] = {0, 0};
    if (!dpk::json::as_int(root.get("ntypes"), &nt) || nt != 2 || !dpk::json::int_list(root.get("sel"), sel, 2) ||
        sel[1] != 92) {
        std::printf("valid header read wrong\n");
        return 1;
    }
    for (size_t n = 0; n < good.size(); ++n)
        if (parse(good.substr(0, n))) { std::printf("truncation at %zu accepted\n", n); return 1; }
    std::mt19937 rng(7);
    const char pool[] = "{}[]\",:\\ 0123456789.eE+-tfnul";
    for (int it = 0; it < 20000; ++it) {
        std::string s = good;
        const int edits = 1 + (int)(rng() % 8);
        for (int e = 0; e < edits; ++e) {
            const size_t at = rng() % (s.size() + 1);
            const int op = (int)(rng() % 3);
            const char ch = rng() % 4 ? pool[rng() % (sizeof(pool) - 1)] : (char)(rng() & 0xff);
            if (op == 0 && at < s.size()) s[at] = ch;
            else if (op == 1) s.insert(s.begin() + (long)at, ch);
            else if (at < s.size()) s.erase(at, 1);
        }
        parse(s);   // any outcome, as long as nothing reads out of bounds
    }
    if (parse(std::string(5000, '[') + std::string(5000, ']'))) { std::printf("deep nesting accepted\n"); return 1; }
    if (parse("{\"a\": " + std::string(3000, '[') + "]}")) { std::printf("unbalanced nesting accepted\n"); return 1; }
    std::printf("json header fuzz ok\n");
    return 0;
}
