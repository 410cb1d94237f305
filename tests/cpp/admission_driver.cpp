// Host test driver for the serving admission logic (csrc/admission.hpp).
// Reads commands from stdin, one per line, and prints one result line each:
//   init S          -> "ok"
//   alloc B         -> offset, or -1 when no free range fits
//   release O B     -> "ok"
//   free            -> "<free bytes> <free ranges>"
//   pick MAXSKIPS B1 B2 ...   (a fresh queue of requests of these sizes,
//                              admitted until pick fails) -> admitted indices
#include <cstdio>
#include <deque>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "admission.hpp"

struct Req {
    size_t bytes;
    int skips;
    int index;
};

int main() {
    jfnk::RangeAllocator ra;
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        std::string cmd;
        in >> cmd;
        if (cmd == "init") {
            size_t s;
            in >> s;
            ra.init(s);
            std::cout << "ok\n";
        } else if (cmd == "alloc") {
            size_t b, off = 0;
            in >> b;
            if (ra.alloc(b, &off)) std::cout << off << "\n";
            else std::cout << -1 << "\n";
        } else if (cmd == "release") {
            size_t o, b;
            in >> o >> b;
            ra.release(o, b);
            std::cout << "ok\n";
        } else if (cmd == "free") {
            std::cout << ra.free_bytes() << " " << ra.free_ranges() << "\n";
        } else if (cmd == "pick") {
            int max_skips;
            in >> max_skips;
            std::vector<Req> reqs;
            size_t b;
            while (in >> b) reqs.push_back(Req{b, 0, (int)reqs.size()});
            std::deque<Req*> q;
            for (auto& r : reqs) q.push_back(&r);
            Req* got = nullptr;
            size_t off = 0;
            std::string out;
            while (jfnk::pick_request(q, ra, max_skips, &got, &off)) out += std::to_string(got->index) + " ";
            std::cout << (out.empty() ? "-" : out) << "\n";
        } else {
            std::cout << "?\n";
        }
        std::cout.flush();
    }
    return 0;
}
