// json_header.h -- the JSON subset of the model file's header: objects, arrays, strings, numbers,
// true/false/null, parsed by recursive descent with a depth limit (host code; the file is input
// the library does not control, so every read is bounded by the buffer's end).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace dpk {
namespace json {

// A JSON value (the subset a header needs: objects, arrays, strings, numbers, true/false/null).
struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    bool b = false;
    double num = 0.0;
    std::string str;
    std::vector<JVal> arr;
    std::map<std::string, JVal> obj;
    const JVal* get(const char* key) const {
        auto it = obj.find(key);
        return kind == OBJ && it != obj.end() ? &it->second : nullptr;
    }
};

struct JParser {
    const char* p;
    const char* end;
    bool ok = true;
    void ws() { while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p; }
    bool lit(const char* w) {
        const size_t n = std::strlen(w);
        if ((size_t)(end - p) < n || std::strncmp(p, w, n) != 0) return false;
        p += n;
        return true;
    }
    JVal value(int depth) {
        JVal v;
        ws();
        if (p >= end || depth > 32) { ok = false; return v; }
        if (*p == '{') {
            v.kind = JVal::OBJ;
            ++p;
            ws();
            if (p < end && *p == '}') { ++p; return v; }
            while (ok) {
                ws();
                JVal k = value(depth + 1);
                if (!ok || k.kind != JVal::STR) { ok = false; break; }
                ws();
                if (p >= end || *p != ':') { ok = false; break; }
                ++p;
                v.obj[k.str] = value(depth + 1);
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == '}') { ++p; break; }
                ok = false;
            }
        } else if (*p == '[') {
            v.kind = JVal::ARR;
            ++p;
            ws();
            if (p < end && *p == ']') { ++p; return v; }
            while (ok) {
                v.arr.push_back(value(depth + 1));
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == ']') { ++p; break; }
                ok = false;
            }
        } else if (*p == '"') {
            v.kind = JVal::STR;
            ++p;
            while (p < end && *p != '"') {
                if (*p == '\\' && p + 1 < end) {
                    ++p;
                    const char e = *p;
                    v.str += e == 'n' ? '\n' : e == 't' ? '\t' : e;   // \" \\ \/ and the rest as is
                } else {
                    v.str += *p;
                }
                ++p;
            }
            if (p >= end) { ok = false; return v; }
            ++p;
        } else if (lit("true")) {
            v.kind = JVal::BOOL;
            v.b = true;
        } else if (lit("false")) {
            v.kind = JVal::BOOL;
        } else if (lit("null")) {
            v.kind = JVal::NUL;
        } else {
            char* q = nullptr;
            std::string tok(p, std::min<size_t>(64, end - p));
            v.num = std::strtod(tok.c_str(), &q);
            if (q == tok.c_str()) { ok = false; return v; }
            v.kind = JVal::NUM;
            p += q - tok.c_str();
        }
        return v;
    }
};

inline bool as_int(const JVal* v, int32_t* out)
{
    if (!v || v->kind != JVal::NUM || v->num != std::floor(v->num) || std::fabs(v->num) > 2e9) return false;
    *out = (int32_t)v->num;
    return true;
}

inline bool as_num(const JVal* v, double* out)
{
    if (!v || v->kind != JVal::NUM) return false;
    *out = v->num;
    return true;
}

inline bool int_list(const JVal* v, int32_t* out, int n)
{
    if (!v || v->kind != JVal::ARR || (int)v->arr.size() != n) return false;
    for (int k = 0; k < n; ++k)
        if (!as_int(&v->arr[k], &out[k])) return false;
    return true;
}

}  // namespace json
}  // namespace dpk
