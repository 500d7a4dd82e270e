// tune_cache.cpp -- reading and writing the sweep-shape tuning cache (format in tune_cache.h).
#include "tune_cache.h"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <vector>

namespace rt3d_tune {

namespace {

// entries in file order: key -> object text
bool read_entries(const std::string &path, std::vector<std::pair<std::string, std::string>> &out)
{
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    while (std::getline(f, line)) {
        size_t a = line.find('"');
        if (a == std::string::npos) continue;
        size_t b = line.find('"', a + 1);
        if (b == std::string::npos) continue;
        size_t colon = line.find(':', b + 1);
        if (colon == std::string::npos) continue;
        std::string val = line.substr(colon + 1);
        while (!val.empty() && (val.back() == ',' || val.back() == ' ' || val.back() == '\r')) val.pop_back();
        while (!val.empty() && val.front() == ' ') val.erase(val.begin());
        if (val.empty() || val.front() != '{' || val.back() != '}') continue;
        out.emplace_back(line.substr(a + 1, b - a - 1), val);
    }
    return true;
}

}  // namespace

bool lookup(const std::string &path, const std::string &key, int &shape)
{
    std::vector<std::pair<std::string, std::string>> e;
    if (path.empty() || !read_entries(path, e)) return false;
    for (const auto &kv : e) {
        if (kv.first != key) continue;
        const size_t p = kv.second.find("\"shape\":");
        if (p == std::string::npos) return false;
        char *end = nullptr;
        const char *s = kv.second.c_str() + p + 8;
        const long v = std::strtol(s, &end, 10);
        if (end == s) return false;
        shape = int(v);
        return true;
    }
    return false;
}

bool store(const std::string &path, const std::string &key, const std::string &entry_json, std::string &err)
{
    if (key.find('"') != std::string::npos) { err = "cache key holds a quote"; return false; }
    std::vector<std::pair<std::string, std::string>> e;
    read_entries(path, e);   // a missing file starts empty
    bool found = false;
    for (auto &kv : e)
        if (kv.first == key) { kv.second = entry_json; found = true; }
    if (!found) e.emplace_back(key, entry_json);
    std::ostringstream os;
    os << "{\n";
    for (size_t i = 0; i < e.size(); ++i)
        os << "\"" << e[i].first << "\": " << e[i].second << (i + 1 < e.size() ? ",\n" : "\n");
    os << "}\n";
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) { err = "cannot write " + tmp; return false; }
        f << os.str();
        if (!f) { err = "cannot write " + tmp; return false; }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) { err = "cannot rename " + tmp; return false; }
    return true;
}

}  // namespace rt3d_tune
