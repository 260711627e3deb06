// TetGen mesh files, the paper's input format (Section 2.2: the Delaunay
// tetrahedralisation comes from TetGen; its .node file lists the points,
// its .ele file the tetrahedra), read on the host.  Host code only: no GPU
// call, so it also runs where no device is present.
//
// .node: a header "<points> <dimension = 3> <attributes> <boundary marker 0|1>",
// then one line per point "<index> <x> <y> <z> [attributes] [marker]".
// .ele:  a header "<tets> <nodes per tet = 4 or 10> <attributes>", then one line
// per tet "<index> <n1> <n2> <n3> <n4> [6 more nodes] [attributes]".
// '#' starts a comment; blank lines are skipped.  The first point index sets
// the numbering base (0 or 1); points must be numbered consecutively from it,
// tets likewise, and every tet node must name a point.  Ten-node tets keep
// their four corners.
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

namespace {

struct Reader {
    FILE* f = nullptr;
    std::string path;
    int64_t line = 0;
    std::vector<std::string> tok;

    explicit Reader(const char* p) : path(p) { f = std::fopen(p, "r"); }
    ~Reader() {
        if (f) std::fclose(f);
    }
    [[noreturn]] void fail(const std::string& what) const {
        throw DecError{DEC_EINVAL, path + ":" + std::to_string(line) + ": " + what};
    }
    // the tokens of the next line that holds any (comments removed); false at the end
    bool next() {
        std::string s;
        char buf[4096];
        while (true) {
            s.clear();
            bool got = false;
            while (std::fgets(buf, sizeof(buf), f)) {
                got = true;
                s += buf;
                if (!s.empty() && s.back() == '\n') break;
            }
            if (!got) return false;
            ++line;
            const size_t hash = s.find('#');
            if (hash != std::string::npos) s.resize(hash);
            tok.clear();
            size_t i = 0;
            while (i < s.size()) {
                while (i < s.size() && (s[i] == ' ' || s[i] == '\t' || s[i] == '\r' || s[i] == '\n' || s[i] == ','))
                    ++i;
                size_t j = i;
                while (j < s.size() && !(s[j] == ' ' || s[j] == '\t' || s[j] == '\r' || s[j] == '\n' || s[j] == ','))
                    ++j;
                if (j > i) tok.push_back(s.substr(i, j - i));
                i = j;
            }
            if (!tok.empty()) return true;
        }
    }
    int64_t integer(size_t k, const char* what) const {
        if (k >= tok.size()) fail(std::string("missing ") + what);
        errno = 0;
        char* end = nullptr;
        const long long v = std::strtoll(tok[k].c_str(), &end, 10);
        if (errno || end == tok[k].c_str() || *end) fail(std::string("bad ") + what + " '" + tok[k] + "'");
        return v;
    }
    double real(size_t k, const char* what) const {
        if (k >= tok.size()) fail(std::string("missing ") + what);
        errno = 0;
        char* end = nullptr;
        const double v = std::strtod(tok[k].c_str(), &end);
        if (errno == ERANGE || end == tok[k].c_str() || *end) fail(std::string("bad ") + what + " '" + tok[k] + "'");
        return v;
    }
};

}  // namespace

extern "C" int dec_tetgen_read(const char* node_path, const char* ele_path, int64_t* V_out, int64_t* T_out,
                               double* xyz, int32_t* tets, int32_t* node_marker) {
    free_error().clear();
    try {
        DEC_REQUIRE(node_path && ele_path, DEC_EINVAL, "NULL file name");
        Reader nr(node_path);
        if (!nr.f) throw DecError{DEC_EINVAL, std::string(node_path) + ": cannot open"};
        if (!nr.next()) nr.fail("no header");
        const int64_t V = nr.integer(0, "point count");
        const int64_t dim = nr.tok.size() > 1 ? nr.integer(1, "dimension") : 3;
        const int64_t nattr = nr.tok.size() > 2 ? nr.integer(2, "attribute count") : 0;
        const int64_t has_marker = nr.tok.size() > 3 ? nr.integer(3, "boundary-marker flag") : 0;
        if (V < 4 || V >= (int64_t(1) << 31)) nr.fail("point count out of range");
        if (dim != 3) nr.fail("dimension must be 3");
        if (nattr < 0 || (has_marker != 0 && has_marker != 1)) nr.fail("bad header");

        Reader er(ele_path);
        if (!er.f) throw DecError{DEC_EINVAL, std::string(ele_path) + ": cannot open"};
        if (!er.next()) er.fail("no header");
        const int64_t T = er.integer(0, "tet count");
        const int64_t npt = er.tok.size() > 1 ? er.integer(1, "nodes per tet") : 4;
        const int64_t eattr = er.tok.size() > 2 ? er.integer(2, "attribute count") : 0;
        if (T < 1 || T >= (int64_t(1) << 31) / 4) er.fail("tet count out of range");
        if (npt != 4 && npt != 10) er.fail("nodes per tet must be 4 or 10");
        if (eattr < 0) er.fail("bad header");
        if (V_out) *V_out = V;
        if (T_out) *T_out = T;
        if (!xyz && !tets && !node_marker) return DEC_OK;

        int64_t base = 0;
        for (int64_t i = 0; i < V; ++i) {
            if (!nr.next()) nr.fail("file ends after " + std::to_string(i) + " of " + std::to_string(V) + " points");
            const int64_t id = nr.integer(0, "point index");
            if (i == 0) {
                if (id != 0 && id != 1) nr.fail("the first point index must be 0 or 1");
                base = id;
            } else if (id != base + i) {
                nr.fail("points must be numbered consecutively");
            }
            const size_t want = 4 + static_cast<size_t>(nattr) + static_cast<size_t>(has_marker);
            if (nr.tok.size() != want) nr.fail("expected " + std::to_string(want) + " fields");
            if (xyz)
                for (int c = 0; c < 3; ++c) xyz[3 * i + c] = nr.real(1 + c, "coordinate");
            else
                for (int c = 0; c < 3; ++c) (void)nr.real(1 + c, "coordinate");
            for (int64_t a = 0; a < nattr; ++a) (void)nr.real(4 + a, "attribute");
            const int64_t mk = has_marker ? nr.integer(4 + nattr, "boundary marker") : 0;
            if (node_marker) node_marker[i] = static_cast<int32_t>(mk);
        }
        if (nr.next()) nr.fail("more points than the header gives");

        for (int64_t t = 0; t < T; ++t) {
            if (!er.next()) er.fail("file ends after " + std::to_string(t) + " of " + std::to_string(T) + " tets");
            const int64_t id = er.integer(0, "tet index");
            if (id != base + t) er.fail("tets must be numbered consecutively from the points' base");
            const size_t want = 1 + static_cast<size_t>(npt) + static_cast<size_t>(eattr);
            if (er.tok.size() != want) er.fail("expected " + std::to_string(want) + " fields");
            for (int k = 0; k < npt; ++k) {
                const int64_t v = er.integer(1 + k, "node index") - base;
                if (v < 0 || v >= V) er.fail("node index out of range");
                if (k < 4 && tets) tets[4 * t + k] = static_cast<int32_t>(v);
            }
            for (int64_t a = 0; a < eattr; ++a) (void)er.real(1 + npt + a, "attribute");
        }
        if (er.next()) er.fail("more tets than the header gives");
    } catch (const DecError& e) {
        free_error() = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        free_error() = "out of host memory";
        return DEC_EINVAL;
    }
    return DEC_OK;
}
