// Persistent autotuner cache: JSON read / write (host only; see tune_cache.h).
#include "tune_cache.h"

#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <sys/stat.h>
#include <unistd.h>

namespace vg {

namespace {

constexpr const char* kFormat = "vgconv-tune-1";

// A small JSON reader: objects, arrays, strings, numbers, true / false /
// null.  Only what the cache file needs is kept: the "format" string and,
// per entry, the numeric fields.
struct Reader {
    const std::string& s;
    size_t i = 0;
    bool ok = true;

    explicit Reader(const std::string& text) : s(text) {}

    void ws() {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\t' || s[i] == '\n' || s[i] == '\r')) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool str(std::string* out) {
        ws();
        if (i >= s.size() || s[i] != '"') return ok = false;
        ++i;
        std::string r;
        while (i < s.size() && s[i] != '"') {
            char c = s[i++];
            if (c == '\\') {
                if (i >= s.size()) return ok = false;
                const char e = s[i++];
                switch (e) {
                    case '"': c = '"'; break;
                    case '\\': c = '\\'; break;
                    case '/': c = '/'; break;
                    case 'n': c = '\n'; break;
                    case 't': c = '\t'; break;
                    default: return ok = false;  // no \u escapes in this file
                }
            }
            r.push_back(c);
        }
        if (i >= s.size()) return ok = false;
        ++i;
        if (out) *out = r;
        return true;
    }
    bool num(double* out) {
        ws();
        const char* b = s.c_str() + i;
        char* e = nullptr;
        errno = 0;
        const double v = std::strtod(b, &e);
        if (e == b || errno != 0 || !std::isfinite(v)) return ok = false;
        i += (size_t)(e - b);
        if (out) *out = v;
        return true;
    }
    bool word(const char* w) {
        ws();
        const std::string t(w);
        if (s.compare(i, t.size(), t) != 0) return ok = false;
        i += t.size();
        return true;
    }
    // Skip any value.
    bool skip(int depth = 0) {
        if (depth > 32) return ok = false;
        ws();
        if (i >= s.size()) return ok = false;
        const char c = s[i];
        if (c == '"') return str(nullptr);
        if (c == '{') {
            ++i;
            if (eat('}')) return true;
            do {
                if (!str(nullptr) || !eat(':') || !skip(depth + 1)) return ok = false;
            } while (eat(','));
            return eat('}') || (ok = false);
        }
        if (c == '[') {
            ++i;
            if (eat(']')) return true;
            do {
                if (!skip(depth + 1)) return ok = false;
            } while (eat(','));
            return eat(']') || (ok = false);
        }
        if (c == 't') return word("true");
        if (c == 'f') return word("false");
        if (c == 'n') return word("null");
        return num(nullptr);
    }
    // An entry: an object of numeric fields (others skipped).
    bool entry(std::map<std::string, double>* fields) {
        if (!eat('{')) return ok = false;
        if (eat('}')) return true;
        do {
            std::string k;
            if (!str(&k) || !eat(':')) return ok = false;
            ws();
            if (i < s.size() && (s[i] == '-' || (s[i] >= '0' && s[i] <= '9'))) {
                double v = 0.0;
                if (!num(&v)) return false;
                (*fields)[k] = v;
            } else if (!skip()) {
                return false;
            }
        } while (eat(','));
        return eat('}') || (ok = false);
    }
};

using Entries = std::map<std::string, std::map<std::string, double>>;

// Parse a whole cache file; false if it is not a cache file of this format.
bool parse(const std::string& text, Entries* entries) {
    Reader r(text);
    std::string format;
    bool have_entries = false;
    if (!r.eat('{')) return false;
    if (!r.eat('}')) {
        do {
            std::string k;
            if (!r.str(&k) || !r.eat(':')) return false;
            if (k == "format") {
                if (!r.str(&format)) return false;
            } else if (k == "entries") {
                if (!r.eat('{')) return false;
                have_entries = true;
                if (!r.eat('}')) {
                    do {
                        std::string key;
                        if (!r.str(&key) || !r.eat(':')) return false;
                        std::map<std::string, double> f;
                        if (!r.entry(&f)) return false;
                        (*entries)[key] = f;
                    } while (r.eat(','));
                    if (!r.eat('}')) return false;
                }
            } else if (!r.skip()) {
                return false;
            }
        } while (r.eat(','));
        if (!r.eat('}')) return false;
    }
    r.ws();
    return r.ok && r.i == text.size() && format == kFormat && have_entries;
}

bool read_file(const std::string& path, std::string* out) {
    std::ifstream in(path, std::ios::binary);
    if (!in) return false;
    std::ostringstream ss;
    ss << in.rdbuf();
    if (!in.good() && !in.eof()) return false;
    *out = ss.str();
    return true;
}

std::string quote(const std::string& k) {
    std::string r = "\"";
    for (char c : k) {
        if (c == '"' || c == '\\') r.push_back('\\');
        if (c == '\n') {
            r += "\\n";
            continue;
        }
        r.push_back(c);
    }
    return r + "\"";
}

bool as_int(const std::map<std::string, double>& f, const char* name, int* out) {
    auto it = f.find(name);
    if (it == f.end()) return false;
    const double v = it->second;
    if (v != std::floor(v) || std::fabs(v) > 1e9) return false;
    *out = (int)v;
    return true;
}

// mkdir -p of the directory part of `path`
void make_parent_dirs(const std::string& path) {
    for (size_t pos = path.find('/', 1); pos != std::string::npos; pos = path.find('/', pos + 1))
        (void)::mkdir(path.substr(0, pos).c_str(), 0755);
}

}  // namespace

std::string tune_cache_path() {
    if (const char* v = std::getenv("VG_TUNE_CACHE")) return std::string(v);
    if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x) return std::string(x) + "/vgconv/tune.json";
    if (const char* h = std::getenv("HOME"); h && *h) return std::string(h) + "/.cache/vgconv/tune.json";
    return "";
}

bool tune_choice_valid(const TuneChoice& c) {
    const bool pad_ok = c.pad_bytes == 0 || c.pad_bytes == 256 || c.pad_bytes == 512 || c.pad_bytes == 1024;
    const bool fs_ok = c.fs_L1 == 0 || (c.fs_L1 >= 2 && c.fs_L1 % 2 == 0 && c.fs_L1 <= 32768);
    return pad_ok && (c.xcd_map == 0 || c.xcd_map == 1) && fs_ok && (c.generic == 0 || c.generic == 1);
}

bool tune_cache_lookup(const std::string& path, const std::string& key, TuneChoice* out) {
    if (path.empty()) return false;
    std::string text;
    if (!read_file(path, &text)) return false;
    Entries entries;
    if (!parse(text, &entries)) return false;
    auto it = entries.find(key);
    if (it == entries.end()) return false;
    TuneChoice c;
    if (!as_int(it->second, "pad_bytes", &c.pad_bytes) || !as_int(it->second, "xcd_map", &c.xcd_map) ||
        !as_int(it->second, "fs_L1", &c.fs_L1) || !as_int(it->second, "generic", &c.generic))
        return false;
    auto ms = it->second.find("ms");
    c.ms = ms != it->second.end() ? ms->second : 0.0;
    if (!tune_choice_valid(c)) return false;
    *out = c;
    return true;
}

bool tune_cache_store(const std::string& path, const std::string& key, const TuneChoice& c) {
    if (path.empty() || !tune_choice_valid(c)) return false;
    Entries entries;
    std::string text;
    if (read_file(path, &text) && !parse(text, &entries)) entries.clear();  // corrupt: start afresh
    auto& f = entries[key];
    f.clear();
    f["pad_bytes"] = c.pad_bytes;
    f["xcd_map"] = c.xcd_map;
    f["fs_L1"] = c.fs_L1;
    f["generic"] = c.generic;
    f["ms"] = c.ms;
    std::ostringstream o;
    o.precision(17);
    o << "{\"format\": " << quote(kFormat) << ",\n \"entries\": {";
    bool first = true;
    for (const auto& kv : entries) {
        o << (first ? "\n  " : ",\n  ") << quote(kv.first) << ": {";
        bool f1 = true;
        for (const auto& fv : kv.second) {
            o << (f1 ? "" : ", ") << quote(fv.first) << ": " << fv.second;
            f1 = false;
        }
        o << "}";
        first = false;
    }
    o << "}}\n";
    make_parent_dirs(path);
    const std::string tmp = path + ".tmp." + std::to_string((long)::getpid());
    {
        std::ofstream out(tmp, std::ios::binary | std::ios::trunc);
        if (!out) return false;
        out << o.str();
        out.flush();
        if (!out) {
            (void)std::remove(tmp.c_str());
            return false;
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        (void)std::remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace vg
