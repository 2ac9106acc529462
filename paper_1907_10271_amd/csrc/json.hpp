// Minimal JSON reader for workload definitions (objects, arrays, numbers,
// strings, true/false/null).  Enough for the configuration files; no
// streaming, no unicode escapes beyond passing them through.
#pragma once

#include <cstdlib>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace mlmc {

struct Json {
  enum Type { Null, Bool, Number, String, Array, Object } type = Null;
  bool b = false;
  double num = 0.0;
  std::string str;
  std::vector<Json> arr;
  std::map<std::string, Json> obj;

  bool has(const std::string &k) const { return type == Object && obj.count(k) && obj.at(k).type != Null; }
  const Json &at(const std::string &k) const {
    auto it = obj.find(k);
    if (type != Object || it == obj.end()) throw std::runtime_error("missing key '" + k + "'");
    return it->second;
  }
  double number(const std::string &k) const {
    const Json &v = at(k);
    if (v.type != Number) throw std::runtime_error("key '" + k + "' is not a number");
    return v.num;
  }
  double number_or(const std::string &k, double d) const { return has(k) ? number(k) : d; }
  std::string string_or(const std::string &k, const std::string &d) const {
    return has(k) && at(k).type == String ? at(k).str : d;
  }
  std::vector<double> numbers(const std::string &k) const {
    const Json &v = at(k);
    if (v.type != Array) throw std::runtime_error("key '" + k + "' is not an array");
    std::vector<double> out;
    for (auto &e : v.arr) {
      if (e.type != Number) throw std::runtime_error("array '" + k + "' holds a non-number");
      out.push_back(e.num);
    }
    return out;
  }
};

class JsonParser {
 public:
  explicit JsonParser(const char *s) : p_(s) {}
  Json parse() {
    Json v = value();
    ws();
    if (*p_) fail("trailing characters");
    return v;
  }

 private:
  const char *p_;
  [[noreturn]] void fail(const char *m) { throw std::runtime_error(std::string("JSON: ") + m); }
  void ws() {
    while (*p_ == ' ' || *p_ == '\n' || *p_ == '\t' || *p_ == '\r') ++p_;
  }
  Json value() {
    ws();
    Json v;
    if (*p_ == '{') {
      v.type = Json::Object;
      ++p_;
      ws();
      if (*p_ == '}') { ++p_; return v; }
      for (;;) {
        ws();
        if (*p_ != '"') fail("expected key");
        std::string k = string();
        ws();
        if (*p_ != ':') fail("expected ':'");
        ++p_;
        v.obj[k] = value();
        ws();
        if (*p_ == ',') { ++p_; continue; }
        if (*p_ == '}') { ++p_; break; }
        fail("expected ',' or '}'");
      }
    } else if (*p_ == '[') {
      v.type = Json::Array;
      ++p_;
      ws();
      if (*p_ == ']') { ++p_; return v; }
      for (;;) {
        v.arr.push_back(value());
        ws();
        if (*p_ == ',') { ++p_; continue; }
        if (*p_ == ']') { ++p_; break; }
        fail("expected ',' or ']'");
      }
    } else if (*p_ == '"') {
      v.type = Json::String;
      v.str = string();
    } else if (!strncmp_(p_, "true")) {
      v.type = Json::Bool; v.b = true; p_ += 4;
    } else if (!strncmp_(p_, "false")) {
      v.type = Json::Bool; p_ += 5;
    } else if (!strncmp_(p_, "null")) {
      p_ += 4;
    } else {
      char *end = nullptr;
      v.num = std::strtod(p_, &end);
      if (end == p_) fail("bad value");
      v.type = Json::Number;
      p_ = end;
    }
    return v;
  }
  static int strncmp_(const char *a, const char *b) {
    while (*b) { if (*a != *b) return 1; ++a; ++b; }
    return 0;
  }
  std::string string() {
    ++p_;
    std::string s;
    while (*p_ && *p_ != '"') {
      if (*p_ == '\\' && p_[1]) { s += p_[1]; p_ += 2; continue; }
      s += *p_++;
    }
    if (*p_ != '"') fail("unterminated string");
    ++p_;
    return s;
  }
};

inline Json parse_json(const char *s) { return JsonParser(s).parse(); }

}  // namespace mlmc
