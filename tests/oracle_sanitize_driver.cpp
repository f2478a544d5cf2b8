// Runs every entry point of the oracle (oracle/oracle.cpp, linked into this
// program) once on inputs read from a directory, and writes the outputs back
// there.  The CPU test suite builds it with AddressSanitizer and
// UndefinedBehaviorSanitizer and compares its outputs with the regular build.
//
// Input files (raw little-endian arrays): meta.txt "N M n C S K nb seed",
// params.bin double [N + M + M N], s.bin int8 [n][N], bonds.bin int32 [nb][2],
// sub.bin int8 [N], chains.bin int8 [C][N], sz0chains.bin int8 [C][N].
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

extern "C" {
void ora_philox4x32_10(const uint32_t* ctr, uint64_t seed, uint32_t* out);
void ora_init_chains(int N, int C, uint64_t seed, int chain_offset, int total_sz_zero, int8_t* out);
void ora_log_psi(int N, int M, const double* params, const int8_t* s, int64_t n, double* out);
void ora_sample(int N, int M, const double* params, int rule, int n_bonds, const int32_t* bonds,
                int C, int S, int K, uint64_t seed, uint64_t prop_base, int chain_offset, int mode,
                int8_t* chains, int8_t* samples, uint8_t* accept_log, double* margins,
                int64_t* n_acc);
void ora_local_energy(int N, int M, const double* params, int kind, int n_bonds,
                      const int32_t* bonds, double J, double h, const int8_t* sub,
                      const int8_t* s, int64_t n, double* out);
void ora_jacobian(int N, int M, const double* params, const int8_t* s, int64_t n, double* O);
}

template <typename T>
static std::vector<T> load(const std::string& path, size_t count) {
    std::vector<T> v(count);
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f || std::fread(v.data(), sizeof(T), count, f) != count) {
        std::fprintf(stderr, "cannot read %s\n", path.c_str());
        std::exit(2);
    }
    std::fclose(f);
    return v;
}

template <typename T>
static void save(const std::string& path, const std::vector<T>& v) {
    FILE* f = std::fopen(path.c_str(), "wb");
    if (!f || std::fwrite(v.data(), sizeof(T), v.size(), f) != v.size()) {
        std::fprintf(stderr, "cannot write %s\n", path.c_str());
        std::exit(2);
    }
    std::fclose(f);
}

int main(int argc, char** argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s DIR\n", argv[0]);
        return 2;
    }
    const std::string d = std::string(argv[1]) + "/";
    int N, M, n, C, S, K, nb;
    unsigned long long seed;
    FILE* f = std::fopen((d + "meta.txt").c_str(), "r");
    if (!f || std::fscanf(f, "%d %d %d %d %d %d %d %llu", &N, &M, &n, &C, &S, &K, &nb, &seed) != 8)
        return 2;
    std::fclose(f);
    const size_t P = (size_t)N + M + (size_t)M * N;
    auto params = load<double>(d + "params.bin", P);
    auto s = load<int8_t>(d + "s.bin", (size_t)n * N);
    auto bonds = load<int32_t>(d + "bonds.bin", 2 * (size_t)nb);
    auto sub = load<int8_t>(d + "sub.bin", N);
    auto chains = load<int8_t>(d + "chains.bin", (size_t)C * N);
    auto zchains = load<int8_t>(d + "sz0chains.bin", (size_t)C * N);

    std::vector<uint32_t> ph(4 * 16);
    for (int k = 0; k < 16; ++k) {
        const uint32_t ctr[4] = {(uint32_t)k * 2654435761u, (uint32_t)k, (uint32_t)(3 * k), 1u};
        ora_philox4x32_10(ctr, seed + k, ph.data() + 4 * k);
    }
    save(d + "out_philox.bin", ph);
    std::vector<int8_t> init((size_t)C * N), initz((size_t)C * N);
    ora_init_chains(N, C, seed, 5, 0, init.data());
    ora_init_chains(N, C, seed, 5, 1, initz.data());
    save(d + "out_init.bin", init);
    save(d + "out_init_sz0.bin", initz);
    std::vector<double> lp(n), et(n), eh(n), O((size_t)n * P);
    ora_log_psi(N, M, params.data(), s.data(), n, lp.data());
    ora_local_energy(N, M, params.data(), 0, nb, bonds.data(), 1.0, 0.7, nullptr, s.data(), n,
                     et.data());
    ora_local_energy(N, M, params.data(), 1, nb, bonds.data(), 1.0, 0.0, sub.data(), s.data(), n,
                     eh.data());
    ora_jacobian(N, M, params.data(), s.data(), n, O.data());
    save(d + "out_logpsi.bin", lp);
    save(d + "out_eloc_tfim.bin", et);
    save(d + "out_eloc_heis.bin", eh);
    save(d + "out_jacobian.bin", O);
    for (int rule = 0; rule < 2; ++rule) {
        for (int mode = 0; mode < 2; ++mode) {
            std::vector<int8_t> ch = rule ? zchains : chains;
            std::vector<int8_t> smp((size_t)C * S * N);
            std::vector<uint8_t> acc((size_t)C * S * K);
            std::vector<double> mg(C);
            std::vector<int64_t> na(C);
            ora_sample(N, M, params.data(), rule, nb, bonds.data(), C, S, K, seed, 7, 3, mode,
                       ch.data(), smp.data(), acc.data(), mg.data(), na.data());
            const std::string tag = std::to_string(rule) + std::to_string(mode);
            save(d + "out_chains" + tag + ".bin", ch);
            save(d + "out_samples" + tag + ".bin", smp);
            save(d + "out_accepts" + tag + ".bin", acc);
            save(d + "out_nacc" + tag + ".bin", na);
        }
    }
    std::printf("ok\n");
    return 0;
}
