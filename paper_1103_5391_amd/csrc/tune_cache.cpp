// Persisted autotuner choices: key construction and a small JSON reader and writer for the
// cache file.  The file holds
//   {"format": "dmrgtst-autotune", "version": 1,
//    "entries": [{"key": "...", "variant": 32, "ms": [10 numbers]}, ...]}
// Numbers are read and written with from_chars / to_chars, so the process locale does not
// change the file.
#include "tune_cache.hpp"

#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <charconv>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>

#include "../../include/dmrgtst.h"
#include "plan.hpp"

namespace dmrg {

namespace {

constexpr const char* kFormat = "dmrgtst-autotune";
constexpr int kVersion = 1;
constexpr int kMaxDepth = 32;                    // nesting the reader accepts
constexpr long kMaxFile = 64L << 20;             // bytes the reader accepts

const char* precision_name(int p) {
    switch (p) {
        case DMRG_FP64: return "fp64";
        case DMRG_FP32: return "fp32";
        case DMRG_BF16X3: return "bf16x3";
        case DMRG_BF16X6: return "bf16x6";
        default: return "unknown";
    }
}

// ---- JSON values and a recursive-descent reader ----

struct JVal {
    enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
    bool b = false;
    double num = 0.0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;

    const JVal* get(const char* name) const {
        for (const auto& kv : obj)
            if (kv.first == name) return &kv.second;
        return nullptr;
    }
};

class Reader {
  public:
    Reader(const char* b, const char* e) : beg_(b), p_(b), end_(e) {}

    bool document(JVal& v) {
        if (!value(v, 0)) return false;
        ws();
        if (p_ != end_) return fail("text after the top-level value");
        return true;
    }
    std::string error() const { return err_; }

  private:
    const char* beg_;
    const char* p_;
    const char* end_;
    std::string err_;

    bool fail(const char* what) {
        if (err_.empty()) err_ = std::string(what) + " at byte " + std::to_string(p_ - beg_);
        return false;
    }
    void ws() {
        while (p_ < end_ && (*p_ == ' ' || *p_ == '\t' || *p_ == '\n' || *p_ == '\r')) ++p_;
    }
    bool lit(const char* word) {
        const size_t n = std::strlen(word);
        if ((size_t)(end_ - p_) < n || std::memcmp(p_, word, n) != 0) return fail("bad literal");
        p_ += n;
        return true;
    }
    bool value(JVal& v, int depth) {
        if (depth > kMaxDepth) return fail("nesting too deep");
        ws();
        if (p_ == end_) return fail("unexpected end");
        switch (*p_) {
            case '{': return object(v, depth);
            case '[': return array(v, depth);
            case '"': v.kind = JVal::Str; return string(v.str);
            case 't': v.kind = JVal::Bool; v.b = true; return lit("true");
            case 'f': v.kind = JVal::Bool; v.b = false; return lit("false");
            case 'n': v.kind = JVal::Null; return lit("null");
            default: v.kind = JVal::Num; return number(v.num);
        }
    }
    bool object(JVal& v, int depth) {
        v.kind = JVal::Obj;
        ++p_;
        ws();
        if (p_ < end_ && *p_ == '}') { ++p_; return true; }
        for (;;) {
            ws();
            if (p_ == end_ || *p_ != '"') return fail("expected a member name");
            std::string name;
            if (!string(name)) return false;
            ws();
            if (p_ == end_ || *p_ != ':') return fail("expected ':'");
            ++p_;
            v.obj.emplace_back(std::move(name), JVal{});
            if (!value(v.obj.back().second, depth + 1)) return false;
            ws();
            if (p_ == end_) return fail("unexpected end in an object");
            if (*p_ == ',') { ++p_; continue; }
            if (*p_ == '}') { ++p_; return true; }
            return fail("expected ',' or '}'");
        }
    }
    bool array(JVal& v, int depth) {
        v.kind = JVal::Arr;
        ++p_;
        ws();
        if (p_ < end_ && *p_ == ']') { ++p_; return true; }
        for (;;) {
            v.arr.emplace_back();
            if (!value(v.arr.back(), depth + 1)) return false;
            ws();
            if (p_ == end_) return fail("unexpected end in an array");
            if (*p_ == ',') { ++p_; continue; }
            if (*p_ == ']') { ++p_; return true; }
            return fail("expected ',' or ']'");
        }
    }
    static void utf8(std::string& s, unsigned cp) {
        if (cp < 0x80) {
            s += (char)cp;
        } else if (cp < 0x800) {
            s += (char)(0xC0 | (cp >> 6));
            s += (char)(0x80 | (cp & 0x3F));
        } else if (cp < 0x10000) {
            s += (char)(0xE0 | (cp >> 12));
            s += (char)(0x80 | ((cp >> 6) & 0x3F));
            s += (char)(0x80 | (cp & 0x3F));
        } else {
            s += (char)(0xF0 | (cp >> 18));
            s += (char)(0x80 | ((cp >> 12) & 0x3F));
            s += (char)(0x80 | ((cp >> 6) & 0x3F));
            s += (char)(0x80 | (cp & 0x3F));
        }
    }
    bool hex4(unsigned& cp) {
        if (end_ - p_ < 4) return fail("short \\u escape");
        cp = 0;
        for (int i = 0; i < 4; ++i, ++p_) {
            const char c = *p_;
            cp <<= 4;
            if (c >= '0' && c <= '9') cp |= (unsigned)(c - '0');
            else if (c >= 'a' && c <= 'f') cp |= (unsigned)(c - 'a' + 10);
            else if (c >= 'A' && c <= 'F') cp |= (unsigned)(c - 'A' + 10);
            else return fail("bad \\u escape");
        }
        return true;
    }
    bool string(std::string& s) {
        ++p_;   // opening quote
        for (;;) {
            if (p_ == end_) return fail("unterminated string");
            const char c = *p_++;
            if (c == '"') return true;
            if ((unsigned char)c < 0x20) return fail("control character in a string");
            if (c != '\\') { s += c; continue; }
            if (p_ == end_) return fail("unterminated escape");
            const char x = *p_++;
            switch (x) {
                case '"': s += '"'; break;
                case '\\': s += '\\'; break;
                case '/': s += '/'; break;
                case 'b': s += '\b'; break;
                case 'f': s += '\f'; break;
                case 'n': s += '\n'; break;
                case 'r': s += '\r'; break;
                case 't': s += '\t'; break;
                case 'u': {
                    unsigned cp;
                    if (!hex4(cp)) return false;
                    if (cp >= 0xD800 && cp < 0xDC00) {   // high surrogate: a low one must follow
                        unsigned lo;
                        if (end_ - p_ < 2 || p_[0] != '\\' || p_[1] != 'u')
                            return fail("unpaired surrogate");
                        p_ += 2;
                        if (!hex4(lo)) return false;
                        if (lo < 0xDC00 || lo >= 0xE000) return fail("unpaired surrogate");
                        cp = 0x10000 + ((cp - 0xD800) << 10) + (lo - 0xDC00);
                    } else if (cp >= 0xDC00 && cp < 0xE000) {
                        return fail("unpaired surrogate");
                    }
                    utf8(s, cp);
                    break;
                }
                default: return fail("bad escape");
            }
        }
    }
    bool number(double& out) {
        // JSON grammar: -? (0 | [1-9][0-9]*) (. [0-9]+)? ([eE] [+-]? [0-9]+)?
        const char* s = p_;
        const char* q = p_;
        auto digits = [&]() {
            const char* d = q;
            while (q < end_ && *q >= '0' && *q <= '9') ++q;
            return q > d;
        };
        if (q < end_ && *q == '-') ++q;
        if (q < end_ && *q == '0') ++q;
        else if (!digits()) return fail("bad number");
        if (q < end_ && *q == '.') {
            ++q;
            if (!digits()) return fail("bad number");
        }
        if (q < end_ && (*q == 'e' || *q == 'E')) {
            ++q;
            if (q < end_ && (*q == '+' || *q == '-')) ++q;
            if (!digits()) return fail("bad number");
        }
        const auto r = std::from_chars(s, q, out);
        if (r.ec != std::errc() || r.ptr != q) return fail("number out of range");
        p_ = q;
        return true;
    }
};

// ---- writer ----

void put_string(std::string& o, const std::string& s) {
    o += '"';
    for (const char c : s) {
        const unsigned char u = (unsigned char)c;
        if (c == '"') o += "\\\"";
        else if (c == '\\') o += "\\\\";
        else if (u < 0x20) {
            char buf[8];
            std::snprintf(buf, sizeof buf, "\\u%04x", u);
            o += buf;
        } else {
            o += c;
        }
    }
    o += '"';
}

void put_number(std::string& o, double v) {
    if (!std::isfinite(v)) v = -1.0;   // JSON has no NaN or infinity: stored as not timed
    char buf[32];
    const auto r = std::to_chars(buf, buf + sizeof buf, v);   // shortest form that reads back
    o.append(buf, r.ptr);
}

std::string serialise(const std::vector<TuneEntry>& es) {
    std::string o = "{\n  \"format\": \"";
    o += kFormat;
    o += "\",\n  \"version\": " + std::to_string(kVersion) + ",\n  \"entries\": [";
    for (size_t i = 0; i < es.size(); ++i) {
        o += i ? ",\n    {\"key\": " : "\n    {\"key\": ";
        put_string(o, es[i].key);
        o += ", \"variant\": " + std::to_string(es[i].variant) + ", \"ms\": [";
        for (int t = 0; t < kTuneTimes; ++t) {
            if (t) o += ", ";
            put_number(o, es[i].ms[t]);
        }
        o += "]}";
    }
    o += es.empty() ? "]\n}\n" : "\n  ]\n}\n";
    return o;
}

bool whole_number(const JVal& v, int& out) {
    if (v.kind != JVal::Num || !(v.num >= -2147483648.0 && v.num <= 2147483647.0)) return false;
    out = (int)v.num;
    return (double)out == v.num;
}

}  // namespace

std::string tune_key(const std::vector<const Plan*>& plans, int precision, const std::string& arch) {
    std::map<int, int64_t> hs, he;
    int64_t terms = 0;
    for (const Plan* P : plans) {
        terms += (int64_t)P->terms.size();
        for (const PsiBlock& b : P->blocks) {
            ++hs[(b.d + kTuneBucket - 1) / kTuneBucket * kTuneBucket];
            ++he[(b.e + kTuneBucket - 1) / kTuneBucket * kTuneBucket];
        }
    }
    std::string k = arch + "/" + precision_name(precision) + "/problems=" +
                    std::to_string(plans.size()) + "/terms=" + std::to_string(terms);
    for (int side = 0; side < 2; ++side) {
        k += side ? "/E=" : "/S=";
        bool first = true;
        for (const auto& kv : side ? he : hs) {
            if (!first) k += ',';
            first = false;
            k += std::to_string(kv.first) + ":" + std::to_string(kv.second);
        }
    }
    return k;
}

std::string tune_cache_read(const std::string& path, std::vector<TuneEntry>& out) {
    out.clear();
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) {
        if (errno == ENOENT) return "";
        return "cannot open the tuning cache " + path + ": " + std::strerror(errno);
    }
    std::string text;
    char buf[65536];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) {
        text.append(buf, got);
        if ((long)text.size() > kMaxFile) {
            std::fclose(f);
            return "tuning cache " + path + " is larger than 64 MiB";
        }
    }
    const bool bad = std::ferror(f) != 0;
    std::fclose(f);
    if (bad) return "cannot read the tuning cache " + path;
    JVal doc;
    Reader rd(text.data(), text.data() + text.size());
    if (!rd.document(doc)) return "tuning cache " + path + " is not JSON: " + rd.error();
    const JVal* fmt = doc.kind == JVal::Obj ? doc.get("format") : nullptr;
    const JVal* ver = doc.kind == JVal::Obj ? doc.get("version") : nullptr;
    int version = 0;
    if (!fmt || fmt->kind != JVal::Str || fmt->str != kFormat || !ver ||
        !whole_number(*ver, version) || version != kVersion)
        return "tuning cache " + path + " is not a version-1 " + kFormat + " file";
    const JVal* ents = doc.get("entries");
    if (!ents || ents->kind != JVal::Arr)
        return "tuning cache " + path + " has no entries array";
    for (const JVal& e : ents->arr) {
        const JVal* k = e.kind == JVal::Obj ? e.get("key") : nullptr;
        const JVal* v = e.kind == JVal::Obj ? e.get("variant") : nullptr;
        const JVal* ms = e.kind == JVal::Obj ? e.get("ms") : nullptr;
        TuneEntry t;
        if (!k || k->kind != JVal::Str || !v || !whole_number(*v, t.variant))
            return "tuning cache " + path + " has an entry without a key or a variant";
        t.key = k->str;
        std::fill(t.ms, t.ms + kTuneTimes, -1.0);
        if (ms) {
            if (ms->kind != JVal::Arr || ms->arr.size() != (size_t)kTuneTimes)
                return "tuning cache " + path + " has an entry whose ms is not 10 numbers";
            for (int i = 0; i < kTuneTimes; ++i) {
                if (ms->arr[i].kind != JVal::Num)
                    return "tuning cache " + path + " has an entry whose ms is not 10 numbers";
                t.ms[i] = ms->arr[i].num;
            }
        }
        out.push_back(std::move(t));
    }
    return "";
}

std::string tune_cache_find(const std::string& path, const std::string& key, TuneEntry& out,
                            bool& found) {
    found = false;
    std::vector<TuneEntry> es;
    std::string err = tune_cache_read(path, es);
    if (!err.empty()) return err;
    for (const TuneEntry& e : es)   // the last entry of a key wins
        if (e.key == key) {
            out = e;
            found = true;
        }
    return "";
}

std::string tune_cache_put(const std::string& path, const TuneEntry& e) {
    std::vector<TuneEntry> es;
    std::string err = tune_cache_read(path, es);
    if (!err.empty()) return err;
    es.erase(std::remove_if(es.begin(), es.end(),
                            [&](const TuneEntry& x) { return x.key == e.key; }),
             es.end());
    es.push_back(e);
    const std::string text = serialise(es);
    // unique per process and per call, so concurrent stores (other processes, other threads)
    // never share a temporary file
    static std::atomic<unsigned> seq{0};
    const std::string tmp = path + ".tmp." + std::to_string((long)getpid()) + "." +
                            std::to_string(seq.fetch_add(1));
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return "cannot write " + tmp + ": " + std::strerror(errno);
    const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size() &&
                    std::fflush(f) == 0;
    if (std::fclose(f) != 0 || !ok) {
        std::remove(tmp.c_str());
        return "cannot write " + tmp;
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        const std::string why = std::strerror(errno);
        std::remove(tmp.c_str());
        return "cannot replace the tuning cache " + path + ": " + why;
    }
    return "";
}

}  // namespace dmrg
