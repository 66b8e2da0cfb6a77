// model_file.cpp -- the model file of libdpk: a versioned JSON header and the FP64 parameter blob.
//
// A frozen model (the paper's C API reads one such file per model, Sec. III.A) holds the
// description of the se_e2_a model (Sec. II.A.1: cut-offs, per-type capacities sel, per-species
// nets; Sec. IV sizes) and its parameters; a compressed model (Sec. II.A.6) records the table's
// stride and range, and the table is rebuilt from the parameters when the file is loaded.
//
// Layout (all integers and floats little-endian):
//   bytes 0..7      the magic "DPKMODEL"
//   bytes 8..15     uint64 H, the length of the JSON header in bytes
//   next H bytes    the JSON header (UTF-8), then zero bytes up to a multiple of 8
//   then            nparams IEEE-754 binary64 values, in the blob layout of include/dpk.h
// Header keys: "format" ("dpk-se_e2_a"), "version" (1), "ntypes", "sel", "rcut", "rcut_smth",
// "embedding", "axis", "fitting", "type_one_side", "descriptor" ("se_e2_a", "se_e2_r", "se_e3";
// absent means se_e2_a), "nparams", "compression" (null or {"stride", "x_max"}). Unknown keys are ignored; a missing key, a wrong type or another format or
// version is DPK_E_INVALID_ARG.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dpk.h"
#include "dpk_launch.h"
#include "json_header.h"

namespace {

using namespace dpk::json;

constexpr char MAGIC[9] = "DPKMODEL";
constexpr int FORMAT_VERSION = 1;

std::string num17(double x)
{
    char b[64];
    std::snprintf(b, sizeof(b), "%.17g", x);
    return b;
}

}  // namespace

using dpk::set_error;

extern "C" {

int dpk_model_save(const dpk_model* m, const char* path)
{
    if (!m || !path) return set_error(DPK_E_INVALID_ARG, "NULL argument");
    dpk_model_desc d;
    double stride = 0.0, xmax = 0.0;
    int rc = dpk_model_describe(m, &d, nullptr, &stride, &xmax);
    if (rc) return rc;
    const int64_t np = dpk_model_param_count(&d);
    std::vector<double> params((size_t)np);
    if ((rc = dpk_model_describe(m, &d, params.data(), nullptr, nullptr))) return rc;
    std::string h = "{\"format\": \"dpk-se_e2_a\", \"version\": " + std::to_string(FORMAT_VERSION);
    h += ", \"ntypes\": " + std::to_string(d.ntypes) + ", \"sel\": [";
    for (int t = 0; t < d.ntypes; ++t) h += (t ? ", " : "") + std::to_string(d.sel[t]);
    h += "], \"rcut\": " + num17(d.rcut) + ", \"rcut_smth\": " + num17(d.rcut_smth);
    h += ", \"embedding\": [" + std::to_string(d.emb[0]) + ", " + std::to_string(d.emb[1]) + ", " +
         std::to_string(d.emb[2]) + "], \"axis\": " + std::to_string(d.axis);
    h += ", \"fitting\": [" + std::to_string(d.fit[0]) + ", " + std::to_string(d.fit[1]) + ", " +
         std::to_string(d.fit[2]) + "], \"type_one_side\": " + (d.type_one_side ? "true" : "false");
    h += ", \"descriptor\": \"";
    h += d.descriptor == DPK_SE_E2_R ? "se_e2_r" : d.descriptor == DPK_SE_E3 ? "se_e3" : "se_e2_a";
    h += "\", \"nparams\": " + std::to_string((long long)np);
    h += ", \"compression\": ";
    h += stride > 0.0 ? "{\"stride\": " + num17(stride) + ", \"x_max\": " + num17(xmax) + "}" : std::string("null");
    h += "}\n";
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(DPK_E_INVALID_ARG, ("cannot open " + std::string(path) + " for writing").c_str());
    const uint64_t hl = h.size();
    uint8_t len[8];
    for (int k = 0; k < 8; ++k) len[k] = (uint8_t)(hl >> (8 * k));
    const size_t pad = (8 - (16 + hl) % 8) % 8;
    const char zeros[8] = {0};
    bool ok = std::fwrite(MAGIC, 1, 8, f) == 8 && std::fwrite(len, 1, 8, f) == 8 &&
              std::fwrite(h.data(), 1, hl, f) == hl && std::fwrite(zeros, 1, pad, f) == pad;
    // binary64 little-endian (the host byte order of every target of this library)
    ok = ok && std::fwrite(params.data(), sizeof(double), params.size(), f) == params.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return set_error(DPK_E_INVALID_ARG, ("write to " + std::string(path) + " failed").c_str());
    return DPK_OK;
}

int dpk_model_load(const char* path, dpk_model** out)
{
    if (!path || !out) return set_error(DPK_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(DPK_E_INVALID_ARG, ("cannot open " + std::string(path)).c_str());
    std::unique_ptr<FILE, int (*)(FILE*)> guard(f, std::fclose);
    char magic[8];
    uint8_t len[8];
    if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, MAGIC, 8) != 0)
        return set_error(DPK_E_INVALID_ARG, "not a dpk model file (magic)");
    if (std::fread(len, 1, 8, f) != 8) return set_error(DPK_E_INVALID_ARG, "truncated model file");
    uint64_t hl = 0;
    for (int k = 0; k < 8; ++k) hl |= (uint64_t)len[k] << (8 * k);
    if (hl == 0 || hl > (1u << 20)) return set_error(DPK_E_INVALID_ARG, "bad header length in model file");
    std::string h(hl, '\0');
    if (std::fread(&h[0], 1, hl, f) != hl) return set_error(DPK_E_INVALID_ARG, "truncated model header");
    JParser jp{h.data(), h.data() + h.size()};
    JVal root = jp.value(0);
    if (!jp.ok || root.kind != JVal::OBJ) return set_error(DPK_E_INVALID_ARG, "model header is not a JSON object");
    const JVal* fmt = root.get("format");
    int32_t ver = 0;
    if (!fmt || fmt->kind != JVal::STR || fmt->str != "dpk-se_e2_a")
        return set_error(DPK_E_INVALID_ARG, "model header: format is not dpk-se_e2_a");
    if (!as_int(root.get("version"), &ver) || ver != FORMAT_VERSION)
        return set_error(DPK_E_INVALID_ARG, "model header: unsupported version");
    dpk_model_desc d;
    std::memset(&d, 0, sizeof(d));
    const JVal* tos = root.get("type_one_side");
    double nparams_d = 0.0;
    if (!as_int(root.get("ntypes"), &d.ntypes) || d.ntypes < 1 || d.ntypes > DPK_MAX_TYPES ||
        !int_list(root.get("sel"), d.sel, d.ntypes) || !as_num(root.get("rcut"), &d.rcut) ||
        !as_num(root.get("rcut_smth"), &d.rcut_smth) || !int_list(root.get("embedding"), d.emb, 3) ||
        !as_int(root.get("axis"), &d.axis) || !int_list(root.get("fitting"), d.fit, 3) || !tos ||
        tos->kind != JVal::BOOL || !as_num(root.get("nparams"), &nparams_d))
        return set_error(DPK_E_INVALID_ARG, "model header: a key is missing or has the wrong type");
    d.type_one_side = tos->b ? 1 : 0;
    // descriptor kind (absent: se_e2_a, the only kind of the first files)
    const JVal* dk = root.get("descriptor");
    if (dk && dk->kind == JVal::STR && dk->str == "se_e2_r") d.descriptor = DPK_SE_E2_R;
    else if (dk && dk->kind == JVal::STR && dk->str == "se_e3") d.descriptor = DPK_SE_E3;
    else if (dk && !(dk->kind == JVal::STR && dk->str == "se_e2_a"))
        return set_error(DPK_E_INVALID_ARG, "model header: descriptor must be se_e2_a, se_e2_r or se_e3");
    const int64_t np = dpk_model_param_count(&d);
    if (np < 1 || (double)np != nparams_d)
        return set_error(DPK_E_INVALID_ARG, "model header: nparams does not match the description");
    const size_t pad = (8 - (16 + hl) % 8) % 8;
    char skip[8];
    if (pad && std::fread(skip, 1, pad, f) != pad) return set_error(DPK_E_INVALID_ARG, "truncated model file");
    std::vector<double> params((size_t)np);
    if (std::fread(params.data(), sizeof(double), params.size(), f) != params.size())
        return set_error(DPK_E_INVALID_ARG, "truncated parameter blob");
    dpk_model* m = nullptr;
    int rc = dpk_model_create(&d, params.data(), np, &m);
    if (rc) return rc;
    const JVal* cmp = root.get("compression");
    if (cmp && cmp->kind == JVal::OBJ) {
        double stride = 0.0, xmax = 0.0;
        if (!as_num(cmp->get("stride"), &stride) || !as_num(cmp->get("x_max"), &xmax)) {
            dpk_model_free(m);
            return set_error(DPK_E_INVALID_ARG, "model header: compression needs stride and x_max");
        }
        if ((rc = dpk_model_tabulate(m, stride, xmax))) {
            dpk_model_free(m);
            return rc;
        }
    } else if (cmp && cmp->kind != JVal::NUL) {
        dpk_model_free(m);
        return set_error(DPK_E_INVALID_ARG, "model header: compression must be null or an object");
    }
    *out = m;
    return DPK_OK;
}

}  // extern "C"
