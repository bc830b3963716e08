"""Writes the stored expected values under tests/golden/ (closed forms only)."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    path = os.path.join(HERE, "image_counts.txt")
    head = [l for l in open(path) if l.startswith("#")]
    with open(path, "w") as f:
        f.writelines(head)
        for K in range(0, 33):
            f.write("%d %d\n" % (K, (2 * K + 1) * (2 * K * K + 2 * K + 3) // 3))


if __name__ == "__main__":
    main()
