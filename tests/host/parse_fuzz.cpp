// Host-only driver for sanitizer runs of the network loader: parses each
// network file given on the command line, then N deterministic mutations of
// it (truncations, byte changes, dropped or repeated lines, extreme numbers,
// stray text).  Every input is handed over in a heap buffer of exactly its
// length, so that a read past the end is caught.  Exits 0 when every
// unmutated file parses and no mutation crashes the parser; the sanitizers
// abort on any memory or undefined-behaviour error.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "network.hpp"

namespace {

struct Lcg {   // 64-bit linear congruential generator (Knuth's MMIX constants)
    uint64_t s;
    uint64_t next() { return s = s * 6364136223846793005ULL + 1442695040888963407ULL; }
    size_t below(size_t n) { return n ? size_t((next() >> 17) % n) : 0; }
};

std::vector<std::string> split_lines(const std::string &t) {
    std::vector<std::string> out;
    std::string cur;
    for (char ch : t) {
        if (ch == '\n') { out.push_back(cur); cur.clear(); }
        else cur.push_back(ch);
    }
    if (!cur.empty()) out.push_back(cur);
    return out;
}

std::string join_lines(const std::vector<std::string> &ls) {
    std::string t;
    for (auto &l : ls) { t += l; t += '\n'; }
    return t;
}

std::string mutate(const std::string &t, Lcg &g) {
    static const char *extremes[] = {"-1", "0", "99999999", "2147483648", "-2147483649", "1e308", "-1e308",
                                     "nan", "inf", "-0", "1e-320", "65535", "65536", "x", ""};
    std::string m = t;
    switch (g.below(6)) {
    case 0:   // truncate
        m.resize(g.below(m.size() + 1));
        break;
    case 1:   // change a byte
        if (!m.empty()) m[g.below(m.size())] = char(32 + g.below(95));
        break;
    case 2: {   // drop a line
        auto ls = split_lines(m);
        if (!ls.empty()) ls.erase(ls.begin() + long(g.below(ls.size())));
        m = join_lines(ls);
        break;
    }
    case 3: {   // repeat a line
        auto ls = split_lines(m);
        if (!ls.empty()) {
            const size_t i = g.below(ls.size());
            ls.insert(ls.begin() + long(i), ls[i]);
        }
        m = join_lines(ls);
        break;
    }
    case 4: {   // replace one whitespace-separated token of a line by an extreme value
        auto ls = split_lines(m);
        if (!ls.empty()) {
            std::string &l = ls[g.below(ls.size())];
            std::vector<std::string> tok;
            std::istringstream is(l);
            for (std::string w; is >> w;) tok.push_back(w);
            if (!tok.empty()) {
                tok[g.below(tok.size())] = extremes[g.below(sizeof(extremes) / sizeof(extremes[0]))];
                l.clear();
                for (size_t k = 0; k < tok.size(); ++k) l += (k ? " " : "") + tok[k];
            }
        }
        m = join_lines(ls);
        break;
    }
    default: {   // stray text
        static const char *junk[] = {"\n", " ", "\t", "#", "end\n", "species 3\n", "reactions 1\n", "\0", "-"};
        const char *j = junk[g.below(sizeof(junk) / sizeof(junk[0]))];
        m.insert(g.below(m.size() + 1), std::string(j, std::strlen(j) ? std::strlen(j) : 1));
        break;
    }
    }
    return m;
}

int parse_exact(const std::string &t, std::string &err, int &S, int &R) {
    std::vector<char> buf(t.begin(), t.end());   // exactly t.size() bytes, no terminator
    abdf::HostNetwork n;
    const int rc = n.parse(buf.empty() ? nullptr : buf.data(), buf.size(), err);
    S = n.S;
    R = n.R;
    return rc;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 3) {
        std::fprintf(stderr, "usage: %s MUTATIONS FILE...\n", argv[0]);
        return 2;
    }
    const int n_mut = std::atoi(argv[1]);
    int bad = 0;
    for (int f = 2; f < argc; ++f) {
        std::ifstream in(argv[f], std::ios::binary);
        std::stringstream ss;
        ss << in.rdbuf();
        const std::string text = ss.str();
        std::string err;
        int S = 0, R = 0;
        const int rc0 = parse_exact(text, err, S, R);
        std::printf("%s: status %d, %d species, %d reactions\n", argv[f], rc0, S, R);
        if (rc0 != 0) {
            std::printf("  unmutated file rejected: %s\n", err.c_str());
            ++bad;
        }
        Lcg g{uint64_t(f) * 0x9E3779B97F4A7C15ULL + 1};
        int counts[8] = {0};
        for (int i = 0; i < n_mut; ++i) {
            std::string m = mutate(text, g);
            if (g.below(4) == 0) m = mutate(m, g);   // sometimes two mutations
            std::string e2;
            int s2 = 0, r2 = 0;
            const int rc = parse_exact(m, e2, s2, r2);
            counts[(rc >= 0 && rc < 7) ? rc : 7] += 1;
        }
        std::printf("  %d mutations, statuses 0..6: %d %d %d %d %d %d %d, other %d\n", n_mut, counts[0], counts[1],
                    counts[2], counts[3], counts[4], counts[5], counts[6], counts[7]);
        if (counts[7] != 0) ++bad;
    }
    return bad == 0 ? 0 : 1;
}
