// exsum_tunecache.hpp -- the batched form's autotune cache file (host only).
//
// The file is JSON of one fixed shape:
//
//   {"version": 1,
//    "entries": {"<batch signature>": {"min_tasks": 16384, "wg_per_cu": 4, "ms": 1.25}, ...}}
//
// parse() reads it with a complete JSON grammar (objects, arrays, strings with
// escapes, numbers, literals), so that nesting, braces inside strings or
// unknown fields cannot shift what is read: an entry keeps its numeric
// fields, anything else in it is skipped.  Text that is not JSON, or JSON of
// another shape or version, is rejected as a whole; the caller then neither
// uses nor rewrites the file.
#pragma once
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>

namespace exs {
namespace tunecache {

using Fields = std::map<std::string, double>;
using Entries = std::map<std::string, Fields>;

class Reader {
  public:
    explicit Reader(const std::string& t) : s_(t) {}

    bool document(Entries* out) {
        bool version_ok = false, have_entries = false;
        ws();
        if (!take('{')) return false;
        ws();
        if (take('}')) return false;  // neither version nor entries
        for (;;) {
            std::string key;
            ws();
            if (!string(&key)) return false;
            ws();
            if (!take(':')) return false;
            ws();
            if (key == "version") {
                double v = 0;
                if (!number(&v)) return false;
                version_ok = v == 1.0;
            } else if (key == "entries") {
                if (!entries(out)) return false;
                have_entries = true;
            } else if (!skip_value(0)) {
                return false;
            }
            ws();
            if (take('}')) break;
            if (!take(',')) return false;
        }
        ws();
        return p_ == s_.size() && version_ok && have_entries;
    }

  private:
    const std::string& s_;
    size_t p_ = 0;
    static constexpr int MAX_DEPTH = 64;

    void ws() {
        while (p_ < s_.size() && (s_[p_] == ' ' || s_[p_] == '\t' || s_[p_] == '\n' || s_[p_] == '\r'))
            ++p_;
    }
    bool take(char c) {
        if (p_ < s_.size() && s_[p_] == c) {
            ++p_;
            return true;
        }
        return false;
    }
    bool literal(const char* w) {
        size_t n = 0;
        while (w[n]) ++n;
        if (s_.compare(p_, n, w) != 0) return false;
        p_ += n;
        return true;
    }
    static int hexval(char c) {
        if (c >= '0' && c <= '9') return c - '0';
        if (c >= 'a' && c <= 'f') return c - 'a' + 10;
        if (c >= 'A' && c <= 'F') return c - 'A' + 10;
        return -1;
    }
    bool hex4(unsigned* v) {
        if (p_ + 4 > s_.size()) return false;
        *v = 0;
        for (int i = 0; i < 4; ++i) {
            const int h = hexval(s_[p_ + i]);
            if (h < 0) return false;
            *v = *v * 16 + (unsigned)h;
        }
        p_ += 4;
        return true;
    }
    static void utf8(unsigned cp, std::string* out) {
        if (cp < 0x80) {
            out->push_back((char)cp);
        } else if (cp < 0x800) {
            out->push_back((char)(0xC0 | (cp >> 6)));
            out->push_back((char)(0x80 | (cp & 0x3F)));
        } else if (cp < 0x10000) {
            out->push_back((char)(0xE0 | (cp >> 12)));
            out->push_back((char)(0x80 | ((cp >> 6) & 0x3F)));
            out->push_back((char)(0x80 | (cp & 0x3F)));
        } else {
            out->push_back((char)(0xF0 | (cp >> 18)));
            out->push_back((char)(0x80 | ((cp >> 12) & 0x3F)));
            out->push_back((char)(0x80 | ((cp >> 6) & 0x3F)));
            out->push_back((char)(0x80 | (cp & 0x3F)));
        }
    }
    // A JSON string, escapes decoded (\uXXXX to UTF-8).
    bool string(std::string* out) {
        if (!take('"')) return false;
        out->clear();
        while (p_ < s_.size()) {
            const char c = s_[p_++];
            if (c == '"') return true;
            if ((unsigned char)c < 0x20) return false;
            if (c != '\\') {
                out->push_back(c);
                continue;
            }
            if (p_ >= s_.size()) return false;
            const char e = s_[p_++];
            switch (e) {
                case '"': out->push_back('"'); break;
                case '\\': out->push_back('\\'); break;
                case '/': out->push_back('/'); break;
                case 'b': out->push_back('\b'); break;
                case 'f': out->push_back('\f'); break;
                case 'n': out->push_back('\n'); break;
                case 'r': out->push_back('\r'); break;
                case 't': out->push_back('\t'); break;
                case 'u': {
                    unsigned cp;
                    if (!hex4(&cp)) return false;
                    if (cp >= 0xD800 && cp < 0xDC00) {  // a surrogate pair
                        unsigned lo;
                        if (!literal("\\u") || !hex4(&lo) || lo < 0xDC00 || lo >= 0xE000)
                            return false;
                        cp = 0x10000 + ((cp - 0xD800) << 10) + (lo - 0xDC00);
                    } else if (cp >= 0xDC00 && cp < 0xE000) {
                        return false;
                    }
                    utf8(cp, out);
                    break;
                }
                default: return false;
            }
        }
        return false;
    }
    // A JSON number (the grammar's form: no leading '+', no leading zeros).
    bool number(double* v) {
        const size_t b = p_;
        take('-');
        if (take('0')) {
        } else if (p_ < s_.size() && s_[p_] >= '1' && s_[p_] <= '9') {
            while (p_ < s_.size() && s_[p_] >= '0' && s_[p_] <= '9') ++p_;
        } else {
            return false;
        }
        if (take('.')) {
            if (!(p_ < s_.size() && s_[p_] >= '0' && s_[p_] <= '9')) return false;
            while (p_ < s_.size() && s_[p_] >= '0' && s_[p_] <= '9') ++p_;
        }
        if (p_ < s_.size() && (s_[p_] == 'e' || s_[p_] == 'E')) {
            ++p_;
            if (!take('+')) take('-');
            if (!(p_ < s_.size() && s_[p_] >= '0' && s_[p_] <= '9')) return false;
            while (p_ < s_.size() && s_[p_] >= '0' && s_[p_] <= '9') ++p_;
        }
        *v = std::strtod(s_.substr(b, p_ - b).c_str(), nullptr);
        return true;
    }
    bool skip_value(int depth) {
        if (depth > MAX_DEPTH || p_ >= s_.size()) return false;
        const char c = s_[p_];
        if (c == '"') {
            std::string tmp;
            return string(&tmp);
        }
        if (c == '{' || c == '[') {
            const char close = c == '{' ? '}' : ']';
            ++p_;
            ws();
            if (take(close)) return true;
            for (;;) {
                ws();
                if (c == '{') {
                    std::string k;
                    if (!string(&k)) return false;
                    ws();
                    if (!take(':')) return false;
                    ws();
                }
                if (!skip_value(depth + 1)) return false;
                ws();
                if (take(close)) return true;
                if (!take(',')) return false;
            }
        }
        if (c == 't') return literal("true");
        if (c == 'f') return literal("false");
        if (c == 'n') return literal("null");
        double v;
        return number(&v);
    }
    bool entries(Entries* out) {
        if (!take('{')) return false;
        ws();
        if (take('}')) return true;
        for (;;) {
            std::string sig;
            ws();
            if (!string(&sig)) return false;
            ws();
            if (!take(':')) return false;
            ws();
            if (!take('{')) return false;
            Fields f;
            ws();
            if (!take('}')) {
                for (;;) {
                    std::string k;
                    ws();
                    if (!string(&k)) return false;
                    ws();
                    if (!take(':')) return false;
                    ws();
                    double v;
                    const size_t at = p_;
                    if (number(&v)) {
                        f[k] = v;
                    } else {
                        p_ = at;
                        if (!skip_value(1)) return false;
                    }
                    ws();
                    if (take('}')) break;
                    if (!take(',')) return false;
                }
            }
            (*out)[sig] = f;
            ws();
            if (take('}')) return true;
            if (!take(',')) return false;
        }
    }
};

// Parse the cache text; false (and *out untouched) when it is not a cache.
inline bool parse(const std::string& text, Entries* out) {
    Entries e;
    Reader r(text);
    if (!r.document(&e)) return false;
    *out = e;
    return true;
}

// JSON string literal of s (bytes from 0x80 up pass through as UTF-8).
inline std::string quote(const std::string& s) {
    std::string o = "\"";
    for (char c : s) {
        if (c == '"' || c == '\\') {
            o.push_back('\\');
            o.push_back(c);
        } else if ((unsigned char)c < 0x20) {
            char b[8];
            std::snprintf(b, sizeof(b), "\\u%04x", (unsigned)(unsigned char)c);
            o += b;
        } else {
            o.push_back(c);
        }
    }
    return o + "\"";
}

inline std::string render(const Entries& m) {
    std::string o = "{\n  \"version\": 1,\n  \"entries\": {\n";
    size_t i = 0;
    for (auto& kv : m) {
        o += "    " + quote(kv.first) + ": {";
        size_t j = 0;
        for (auto& f : kv.second) {
            char b[64];
            std::snprintf(b, sizeof(b), "%.17g", f.second);
            o += quote(f.first) + ": " + b + (++j < kv.second.size() ? ", " : "");
        }
        o += (++i < m.size()) ? "},\n" : "}\n";
    }
    return o + "  }\n}\n";
}

}  // namespace tunecache
}  // namespace exs
