// tune_cache.h -- the sweep-shape tuning cache: a JSON object, one entry per line,
//   "<device>|<precision>|<grid>": {"shape": s, "threads": t, "lines": l, "ms": [..]}
// Keys hold no quotes.  Entries are replaced in place; the file is rewritten through a temporary
// file and a rename, so a reader never sees half of it.
#pragma once

#include <string>

namespace rt3d_tune {

// Shape index stored for key, or false when the file or the entry is missing or unreadable.
bool lookup(const std::string &path, const std::string &key, int &shape);

// Insert or replace the entry for key (entry_json is the object after the colon).
bool store(const std::string &path, const std::string &key, const std::string &entry_json, std::string &err);

}  // namespace rt3d_tune
