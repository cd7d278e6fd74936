// Tuned launch shapes from the shape tuner's JSON cache, for C callers.
//
// The cache (written by the package's autotune module) maps a device key
//   "cc<major>.<minor>-<CUs>cu|hip<runtime version>"
// to entries keyed by workload class.  The entries this loader reads are
//   "snapshot|p<page size>|b<k>"  single snapshots of that page size whose
//                                  scanned bytes N satisfy 2^k <= N < 2^(k+1)
//   "plan|b<k>"                   plans whose requests scan 2^k..2^(k+1) bytes
// each holding {"params": {"<name>": <integer>, ...}, ...}; other keys and
// fields are skipped.  Parameter names are those of the tuner (diff_blocks,
// pack_blocks, chunk_bytes, ...), each mapped to its CRUM_PARAM_* value.
//
// Host code only: no HIP call is made.
#include "crum.h"
#include "crum_internal.h"

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

namespace crum {

namespace {

// A small recursive-descent reader of the JSON subset the cache uses
// (objects, arrays, strings without unicode escapes, numbers, true, false,
// null).  Values other than objects and integers are parsed and dropped.
struct Reader {
    const char* p;
    const char* end;
    bool ok = true;
    int depth = 0;  // nesting of skipped values, bounded so that input cannot exhaust the stack
    static constexpr int kMaxDepth = 64;

    void ws()
    {
        while (p < end && std::isspace((unsigned char)*p))
            ++p;
    }
    bool eat(char c)
    {
        ws();
        if (p < end && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string* out)
    {
        ws();
        if (p >= end || *p != '"')
            return ok = false;
        ++p;
        std::string s;
        while (p < end && *p != '"') {
            if (*p == '\\') {
                if (++p >= end)
                    return ok = false;
                const char e = *p;
                s.push_back(e == 'n' ? '\n' : e == 't' ? '\t' : e);
            } else {
                s.push_back(*p);
            }
            ++p;
        }
        if (p >= end)
            return ok = false;
        ++p;
        if (out)
            *out = std::move(s);
        return true;
    }
    // a number; *is_int tells whether it was a plain non-negative integer
    bool num(uint64_t* v, bool* is_int)
    {
        ws();
        const char* s = p;
        bool integer = true;
        if (p < end && (*p == '-' || *p == '+')) {
            integer = false;
            ++p;
        }
        while (p < end && (std::isdigit((unsigned char)*p) || *p == '.' || *p == 'e' ||
                           *p == 'E' || *p == '-' || *p == '+')) {
            if (!std::isdigit((unsigned char)*p))
                integer = false;
            ++p;
        }
        if (p == s)
            return ok = false;
        *is_int = integer;
        *v = integer ? std::strtoull(std::string(s, p).c_str(), nullptr, 10) : 0;
        return true;
    }
    bool word(const char* w)
    {
        const size_t n = std::strlen(w);
        if ((size_t)(end - p) >= n && std::strncmp(p, w, n) == 0) {
            p += n;
            return true;
        }
        return ok = false;
    }
    // skip any value
    bool skip()
    {
        ws();
        if (p >= end)
            return ok = false;
        if (*p == '{' || *p == '[') {
            if (depth >= kMaxDepth)
                return ok = false;
            ++depth;
            const bool r = skip_container();
            --depth;
            return r;
        }
        if (*p == '"')
            return str(nullptr);
        if (*p == 't')
            return word("true");
        if (*p == 'f')
            return word("false");
        if (*p == 'n')
            return word("null");
        uint64_t v;
        bool i;
        return num(&v, &i);
    }
    // an object or array (at *p)
    bool skip_container()
    {
        if (*p++ == '{') {
            if (eat('}'))
                return true;
            do {
                if (!str(nullptr) || !eat(':') || !skip())
                    return ok = false;
            } while (eat(','));
            return eat('}') || (ok = false);
        }
        if (eat(']'))
            return true;
        do {
            if (!skip())
                return ok = false;
        } while (eat(','));
        return eat(']') || (ok = false);
    }
    // {"name": integer, ...}: integer members only
    bool int_members(std::vector<std::pair<std::string, uint64_t>>* out)
    {
        if (!eat('{'))
            return ok = false;
        if (eat('}'))
            return true;
        do {
            std::string k;
            if (!str(&k) || !eat(':'))
                return ok = false;
            ws();
            if (p < end && (std::isdigit((unsigned char)*p) || *p == '-')) {
                uint64_t v;
                bool is_int;
                if (!num(&v, &is_int))
                    return false;
                if (is_int)
                    out->emplace_back(k, v);
            } else if (!skip()) {
                return false;
            }
        } while (eat(','));
        return eat('}') || (ok = false);
    }
};

int param_id(const std::string& name)
{
    static const std::pair<const char*, int> names[] = {
        {"diff_blocks", CRUM_PARAM_DIFF_BLOCKS},
        {"pack_blocks", CRUM_PARAM_PACK_BLOCKS},
        {"chunk_bytes", CRUM_PARAM_CHUNK_BYTES},
        {"chunk_max_bytes", CRUM_PARAM_CHUNK_MAX_BYTES},
        {"eager", CRUM_PARAM_EAGER},
        {"drain_chunk_bytes", CRUM_PARAM_DRAIN_CHUNK_BYTES},
        {"diff_unit_shift", CRUM_PARAM_DIFF_UNIT_SHIFT},
        {"diff_nontemporal", CRUM_PARAM_DIFF_NONTEMPORAL},
        {"piece_shift", CRUM_PARAM_PIECE_SHIFT},
        {"pack_depth", CRUM_PARAM_PACK_DEPTH},
        {"diff_priority", CRUM_PARAM_DIFF_PRIORITY},
        {"crc_variant", CRUM_PARAM_CRC_VARIANT},
        {"plan_order", CRUM_PARAM_PLAN_ORDER},
        {"direct_bytes", CRUM_PARAM_DIRECT_BYTES},
        {"chunk_growth", CRUM_PARAM_CHUNK_GROWTH},
        {"pack_nt_store", CRUM_PARAM_PACK_NT_STORE},
        {"pack_prefetch", CRUM_PARAM_PACK_PREFETCH},
        {"pack_nt_load", CRUM_PARAM_PACK_NT_LOAD},
        {"diff_group", CRUM_PARAM_DIFF_GROUP},
    };
    for (const auto& n : names)
        if (name == n.first)
            return n.second;
    return 0;
}

// "snapshot|p65536|b34" or "plan|b36"
bool parse_class(const std::string& key, TunedClass* c)
{
    unsigned long long ps = 0, b = 0;
    char tail = 0;
    if (std::sscanf(key.c_str(), "snapshot|p%llu|b%llu%c", &ps, &b, &tail) == 2) {
        c->kind = 0;
        c->page_size = (uint32_t)ps;
        c->log2_bytes = (uint32_t)b;
        return page_size_ok(ps) && b < 64;
    }
    if (std::sscanf(key.c_str(), "plan|b%llu%c", &b, &tail) == 1) {
        c->kind = 1;
        c->page_size = 0;
        c->log2_bytes = (uint32_t)b;
        return b < 64;
    }
    return false;
}

}  // namespace

int tune_load(const char* path, const std::string& device_key, std::vector<TunedClass>* out)
{
    out->clear();
    FILE* f = std::fopen(path, "rb");
    if (!f)
        return CRUM_EINVAL;
    std::string text;
    char buf[65536];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0)
        text.append(buf, n);
    std::fclose(f);
    Reader r{text.data(), text.data() + text.size()};
    if (!r.eat('{'))
        return CRUM_EINVAL;
    if (r.eat('}'))
        return CRUM_OK;
    do {
        std::string dev;
        if (!r.str(&dev) || !r.eat(':'))
            return CRUM_EINVAL;
        if (dev != device_key) {
            if (!r.skip())
                return CRUM_EINVAL;
            continue;
        }
        if (!r.eat('{'))
            return CRUM_EINVAL;
        if (r.eat('}'))
            continue;
        do {
            std::string cls;
            if (!r.str(&cls) || !r.eat(':'))
                return CRUM_EINVAL;
            TunedClass tc;
            if (!parse_class(cls, &tc)) {
                if (!r.skip())
                    return CRUM_EINVAL;
                continue;
            }
            // the entry: find its "params" member
            if (!r.eat('{'))
                return CRUM_EINVAL;
            bool have = false;
            if (!r.eat('}')) {
                do {
                    std::string k;
                    if (!r.str(&k) || !r.eat(':'))
                        return CRUM_EINVAL;
                    if (k == "params") {
                        std::vector<std::pair<std::string, uint64_t>> kv;
                        if (!r.int_members(&kv))
                            return CRUM_EINVAL;
                        for (auto& e : kv) {
                            const int id = param_id(e.first);
                            if (id)
                                tc.params.emplace_back(id, e.second);
                        }
                        have = true;
                    } else if (!r.skip()) {
                        return CRUM_EINVAL;
                    }
                } while (r.eat(','));
                if (!r.eat('}'))
                    return CRUM_EINVAL;
            }
            if (have)
                out->push_back(std::move(tc));
        } while (r.eat(','));
        if (!r.eat('}'))
            return CRUM_EINVAL;
    } while (r.eat(','));
    if (!r.eat('}'))
        return CRUM_EINVAL;
    return r.ok ? CRUM_OK : CRUM_EINVAL;
}

const TunedClass* tune_find(const std::vector<TunedClass>& v, int kind, uint32_t page_size,
                            uint64_t bytes)
{
    if (v.empty() || bytes == 0)
        return nullptr;
    uint32_t k = 0;
    while (k < 63 && (bytes >> (k + 1)))
        ++k;
    for (const TunedClass& c : v)
        if (c.kind == kind && (kind == 1 || c.page_size == page_size) && c.log2_bytes == k)
            return &c;
    return nullptr;
}

}  // namespace crum
