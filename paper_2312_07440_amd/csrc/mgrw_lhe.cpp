// Les Houches event files: the input and output of the reweighting procedure
// (Sec. 3.2 steps 2 and 8; the paper's outlook, Sec. 5, describes a C++ LHE
// library written for the same purpose).  Host code only.
//
// Reading keeps the file's text: each event block is split into its header
// line, its particle lines and whatever follows them (optional blocks such as
// an existing <rwgt>), so that writing reproduces every byte of the input
// and only adds the new weights.  Momenta are handed out in the structure-of-
// arrays layout of the device kernels, in the process's particle order,
// boosted along the beam axis to the partonic centre-of-mass frame (the frame
// in which the amplitudes' polarisation vectors are defined).
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/mgrw.h"

namespace mgrw {
mgrw_status set_error(mgrw_status code, const std::string& msg);   // mgrw_abi.hip
}

namespace {

struct lhe_particle {
    int id, status;
    double p[5];   // px py pz E m
};

struct lhe_event {
    std::string head;                    // the "<event...>" line and the event header line
    std::vector<std::string> lines;      // particle lines as read
    std::string tail;                    // lines after the particles, before the closing line
    std::string close;                   // the line holding "</event>"
    std::string gap;                     // text up to the next event (the file's end for the last)
    std::vector<lhe_particle> parts;
    double weight;
};

}  // namespace

struct mgrw_lhe {
    std::string prologue;      // everything before the first event
    std::vector<lhe_event> events;
};

namespace {

mgrw_status lhe_fail(mgrw_status code, const std::string& msg) { return mgrw::set_error(code, msg); }

bool starts_with_tag(const std::string& line, const char* tag) {
    size_t i = line.find_first_not_of(" \t\r");
    return i != std::string::npos && line.compare(i, std::strlen(tag), tag) == 0;
}

bool parse_doubles(const std::string& s, double* out, int n) {
    const char* c = s.c_str();
    for (int i = 0; i < n; ++i) {
        char* end = nullptr;
        errno = 0;
        out[i] = std::strtod(c, &end);
        if (end == c || errno == ERANGE) return false;
        c = end;
    }
    return true;
}

// Expected particles of a process in its momentum order: PDG id and
// status (-1 incoming, +1 outgoing).
bool process_signature(int proc, std::vector<int>& ids) {
    switch (proc) {
        case MGRW_EE_MUMU: ids = {-11, 11, -13, 13}; return true;
        case MGRW_GG_TT: ids = {21, 21, 6, -6}; return true;
        case MGRW_GG_TTG: ids = {21, 21, 6, -6, 21}; return true;
        case MGRW_GG_TTGG: ids = {21, 21, 6, -6, 21, 21}; return true;
        case MGRW_GG_TTGGG: ids = {21, 21, 6, -6, 21, 21, 21}; return true;
        case MGRW_EE_5A: ids = {-11, 11, 22, 22, 22, 22, 22}; return true;
        default: return false;
    }
}

}  // namespace

extern "C" {

mgrw_status mgrw_lhe_open(const char* path, mgrw_lhe** out) {
    if (!path || !out) return lhe_fail(MGRW_ERR_ARG, "path or out is NULL");
    *out = nullptr;
    std::ifstream f(path, std::ios::binary);
    if (!f) return lhe_fail(MGRW_ERR_ARG, std::string("cannot open ") + path);
    mgrw_lhe* h = new (std::nothrow) mgrw_lhe;
    if (!h) return lhe_fail(MGRW_ERR_ALLOC, "out of host memory");
    std::string line;
    long lineno = 0;
    enum { OUTSIDE, HEAD, PARTS, TAIL } state = OUTSIDE;
    int nup = 0;
    lhe_event ev;
    auto bad = [&](const std::string& what) {
        delete h;
        return lhe_fail(MGRW_ERR_ARG, std::string(path) + ":" + std::to_string(lineno) + ": " + what);
    };
    while (std::getline(f, line)) {
        ++lineno;
        const std::string text = line + (f.eof() ? "" : "\n");
        switch (state) {
            case OUTSIDE:
                if (starts_with_tag(line, "<event")) {
                    ev = lhe_event();
                    ev.head = text;
                    state = HEAD;
                } else if (h->events.empty()) {
                    h->prologue += text;
                } else {
                    h->events.back().gap += text;
                }
                break;
            case HEAD: {
                double v[6];
                if (!parse_doubles(line, v, 6)) return bad("event header line expected");
                nup = int(v[0]);
                if (nup < 1 || nup > 64 || double(nup) != v[0]) return bad("bad particle count");
                ev.weight = v[2];
                ev.head += text;
                state = PARTS;
                break;
            }
            case PARTS: {
                double v[13];
                if (!parse_doubles(line, v, 13)) return bad("particle line expected");
                lhe_particle q;
                q.id = int(v[0]);
                q.status = int(v[1]);
                for (int i = 0; i < 5; ++i) q.p[i] = v[6 + i];
                ev.parts.push_back(q);
                ev.lines.push_back(text);
                if (int(ev.parts.size()) == nup) state = TAIL;
                break;
            }
            case TAIL:
                if (line.find("</event>") != std::string::npos) {
                    ev.close = text;
                    h->events.push_back(std::move(ev));
                    state = OUTSIDE;
                } else if (starts_with_tag(line, "<event")) {
                    return bad("unterminated event");
                } else {
                    ev.tail += text;
                }
                break;
        }
    }
    if (state != OUTSIDE) return bad("file ends inside an event");
    *out = h;
    return MGRW_OK;
}

mgrw_status mgrw_lhe_info(const mgrw_lhe* h, int64_t* n_events) {
    if (!h || !n_events) return lhe_fail(MGRW_ERR_ARG, "handle or n_events is NULL");
    *n_events = int64_t(h->events.size());
    return MGRW_OK;
}

mgrw_status mgrw_lhe_events(const mgrw_lhe* h, int proc, double* mom, double* w) {
    if (!h || !mom) return lhe_fail(MGRW_ERR_ARG, "handle or mom is NULL");
    std::vector<int> ids;
    if (!process_signature(proc, ids)) return lhe_fail(MGRW_ERR_ARG, "unknown process");
    const int next = int(ids.size());
    const int64_t n = int64_t(h->events.size());
    for (int64_t e = 0; e < n; ++e) {
        const lhe_event& ev = h->events[size_t(e)];
        // assign the event's incoming and outgoing particles to the slots of
        // the process in order of appearance
        int slot_of[64];
        std::vector<bool> used(size_t(next), false);
        int placed = 0;
        for (size_t i = 0; i < ev.parts.size(); ++i) {
            slot_of[i] = -1;
            const lhe_particle& q = ev.parts[i];
            if (q.status != -1 && q.status != 1) continue;   // intermediate or other
            const int first = q.status == -1 ? 0 : 2, last = q.status == -1 ? 2 : next;
            for (int s = first; s < last; ++s)
                if (!used[size_t(s)] && ids[size_t(s)] == q.id) {
                    used[size_t(s)] = true;
                    slot_of[i] = s;
                    ++placed;
                    break;
                }
            if (slot_of[i] < 0)
                return lhe_fail(MGRW_ERR_ARG, "event " + std::to_string(e) + ": particle " + std::to_string(q.id) +
                                                  " (status " + std::to_string(q.status) +
                                                  ") does not belong to the process");
        }
        if (placed != next)
            return lhe_fail(MGRW_ERR_ARG, "event " + std::to_string(e) + ": particle content does not match");
        // longitudinal boost to the frame where the incoming momenta sum to zero
        double E = 0.0, Pz = 0.0, Px = 0.0, Py = 0.0;
        for (size_t i = 0; i < ev.parts.size(); ++i)
            if (slot_of[i] >= 0 && slot_of[i] < 2) {
                Px += ev.parts[i].p[0];
                Py += ev.parts[i].p[1];
                Pz += ev.parts[i].p[2];
                E += ev.parts[i].p[3];
            }
        if (std::fabs(Px) > 1e-9 * E || std::fabs(Py) > 1e-9 * E)
            return lhe_fail(MGRW_ERR_ARG, "event " + std::to_string(e) + ": incoming partons not along the beam axis");
        const double beta = Pz / E, gamma = 1.0 / std::sqrt((1.0 - beta) * (1.0 + beta));
        for (size_t i = 0; i < ev.parts.size(); ++i) {
            const int s = slot_of[i];
            if (s < 0) continue;
            const double* p = ev.parts[i].p;
            const double en = gamma * (p[3] - beta * p[2]);
            const double pz = gamma * (p[2] - beta * p[3]);
            const double v[4] = {en, p[0], p[1], pz};
            for (int m = 0; m < 4; ++m) mom[(int64_t(s) * 4 + m) * n + e] = v[m];
        }
        if (w) w[e] = ev.weight;
    }
    return MGRW_OK;
}

mgrw_status mgrw_lhe_write(const mgrw_lhe* h, const char* path, const double* w_new, int n_points,
                           const char* const* ids) {
    if (!h || !path) return lhe_fail(MGRW_ERR_ARG, "handle or path is NULL");
    if (n_points < 0 || (n_points > 0 && (!w_new || !ids))) return lhe_fail(MGRW_ERR_ARG, "weights or ids missing");
    for (int k = 0; k < n_points; ++k)
        if (!ids[k] || !ids[k][0] || std::strpbrk(ids[k], "'\"<>&\n"))
            return lhe_fail(MGRW_ERR_ARG, "weight ids must be non-empty and free of quotes, markup and newlines");
    // declare the new weights in the header (LHE 3.0 <initrwgt>), if there is one
    std::string prologue = h->prologue;
    if (n_points > 0) {
        std::string decl;
        for (int k = 0; k < n_points; ++k) decl += std::string("<weight id='") + ids[k] + "'> </weight>\n";
        size_t at = prologue.find("</initrwgt>");
        if (at != std::string::npos) {
            prologue.insert(at, decl);
        } else if ((at = prologue.find("</header>")) != std::string::npos) {
            prologue.insert(at, "<initrwgt>\n" + decl + "</initrwgt>\n");
        }
    }
    const std::string tmp = std::string(path) + ".part";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return lhe_fail(MGRW_ERR_ARG, std::string("cannot write ") + tmp);
    const int64_t n = int64_t(h->events.size());
    bool ok = std::fwrite(prologue.data(), 1, prologue.size(), f) == prologue.size();
    char buf[64];
    for (int64_t e = 0; e < n && ok; ++e) {
        const lhe_event& ev = h->events[size_t(e)];
        std::string s = ev.head;
        for (const std::string& l : ev.lines) s += l;
        std::string tail = ev.tail;
        if (n_points > 0) {
            std::string add;
            for (int k = 0; k < n_points; ++k) {
                std::snprintf(buf, sizeof buf, "%.17e", w_new[int64_t(k) * n + e]);
                add += std::string("<wgt id='") + ids[k] + "'> " + buf + " </wgt>\n";
            }
            const size_t close = tail.find("</rwgt>");
            if (close != std::string::npos)
                tail.insert(close, add);   // extend the event's existing block
            else
                tail += "<rwgt>\n" + add + "</rwgt>\n";
        }
        s += tail + ev.close + ev.gap;
        ok = std::fwrite(s.data(), 1, s.size(), f) == s.size();
    }
    if (std::fclose(f) != 0) ok = false;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return lhe_fail(MGRW_ERR_ARG, std::string("writing ") + path + " failed");
    }
    return MGRW_OK;
}

void mgrw_lhe_close(mgrw_lhe* h) { delete h; }

}  // extern "C"
