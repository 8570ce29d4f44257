// Host driver for the autotune cache reader: reads a file, prints what the
// library would take from it.  Built and run by test_tunecache.py.
#include <fstream>
#include <iostream>
#include <sstream>

#include "exsum_tunecache.hpp"

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    std::ifstream f(argv[1], std::ios::binary);
    std::stringstream ss;
    ss << f.rdbuf();
    exs::tunecache::Entries e;
    if (!exs::tunecache::parse(ss.str(), &e)) {
        std::cout << "REJECT\n";
        return 0;
    }
    if (argc > 2) {  // round trip: render what was read, parse it again
        exs::tunecache::Entries e2;
        if (!exs::tunecache::parse(exs::tunecache::render(e), &e2) || e2 != e) {
            std::cout << "ROUNDTRIP-MISMATCH\n";
            return 1;
        }
    }
    std::cout << "OK " << e.size() << "\n";
    for (auto& kv : e) {
        std::cout << kv.first;
        for (auto& fv : kv.second) std::cout << " " << fv.first << "=" << fv.second;
        std::cout << "\n";
    }
    return 0;
}
