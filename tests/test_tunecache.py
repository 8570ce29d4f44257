"""Host tests of the batched form's autotune cache reader (no GPU): the
library's parser is compiled with g++ into a small driver and fed valid
caches, caches with foreign content, and text that is not a cache."""
import json
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2106_00124_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("tc") / "tunecache_driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "tunecache_driver.cpp"), "-o", out], check=True)
    return out


def _read(driver, tmp_path, text, roundtrip=True):
    p = tmp_path / "cache.json"
    p.write_bytes(text.encode() if isinstance(text, str) else text)
    args = [driver, str(p)] + (["rt"] if roundtrip else [])
    r = subprocess.run(args, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.splitlines()
    if lines[0] == "REJECT":
        return None
    entries = {}
    for ln in lines[1:]:
        sig, *fields = ln.split(" ")
        entries[sig] = {k: float(v) for k, v in (f.split("=") for f in fields)}
    assert int(lines[0].split()[1]) == len(entries)
    return entries


def test_written_form_is_read(driver, tmp_path):
    text = ('{\n  "version": 1,\n  "entries": {\n'
            '    "batch-00ff-n7": {"min_tasks": 16384, "wg_per_cu": 4, "ms": 1.25},\n'
            '    "batch-0a0b-n2": {"min_tasks": 4096, "wg_per_cu": 8, "ms": 0.5}\n  }\n}\n')
    e = _read(driver, tmp_path, text)
    assert e == {"batch-00ff-n7": {"min_tasks": 16384, "wg_per_cu": 4, "ms": 1.25},
                 "batch-0a0b-n2": {"min_tasks": 4096, "wg_per_cu": 8, "ms": 0.5}}


def test_python_json_dump_is_read(driver, tmp_path):
    doc = {"entries": {"batch-1-n1": {"wg_per_cu": 2, "min_tasks": 65536}}, "version": 1}
    assert _read(driver, tmp_path, json.dumps(doc)) == {
        "batch-1-n1": {"min_tasks": 65536, "wg_per_cu": 2}}


def test_nested_and_foreign_fields_do_not_shift_entries(driver, tmp_path):
    # braces inside strings, nested objects and arrays, extra top-level keys:
    # a substring scan would take the wrong braces here
    doc = {"note": "a } brace { and \"batch-evil\": {\"min_tasks\": 1}",
           "version": 1,
           "entries": {
               "batch-a-n3": {"meta": {"tiles": [1, {"x": "}"}], "s": "{"},
                              "min_tasks": 4096, "wg_per_cu": 2, "ok": True},
               "batch-b-n4": {"min_tasks": 1.5e4, "wg_per_cu": 8, "tag": None}},
           "other": [[[]], {}, "batch-c-n5"]}
    assert _read(driver, tmp_path, json.dumps(doc)) == {
        "batch-a-n3": {"min_tasks": 4096, "wg_per_cu": 2},
        "batch-b-n4": {"min_tasks": 15000, "wg_per_cu": 8}}


def test_escapes_in_keys(driver, tmp_path):
    doc = {"version": 1, "entries": {"batch-é\"\\-n1": {"min_tasks": 1, "wg_per_cu": 1}}}
    for ensure_ascii in (True, False):
        e = _read(driver, tmp_path, json.dumps(doc, ensure_ascii=ensure_ascii))
        assert list(e) == ["batch-é\"\\-n1"]


@pytest.mark.parametrize("text", [
    "",                                          # empty file
    "not json",
    '{"version": 1}',                            # no entries
    '{"entries": {}}',                           # no version
    '{"version": 2, "entries": {}}',             # another version
    '{"version": "1", "entries": {}}',
    '{"version": 1, "entries": []}',             # entries not an object
    '{"version": 1, "entries": {"batch-x": 3}}',  # entry not an object
    '{"version": 1, "entries": {"batch-x": {"min_tasks": 1,}}}',  # trailing comma
    '{"version": 1, "entries": {}} trailing',
    '{"version": 1, "entries": {"batch-x": {"min_tasks": 01}}}',  # leading zero
    '{"version": 1, "entries": {"batch-\\x": {}}}',              # bad escape
    '{"version": 1, "entries": {"batch-\\ud800": {}}}',          # lone surrogate
    '{"version": 1, "entries": {"batch-x": {"a": [1, 2}}}',      # unbalanced
    '{"version": 1, "entries": {"b": {"x": ' + '[' * 100 + ']' * 100 + '}}}',  # too deep
])
def test_non_cache_text_is_rejected(driver, tmp_path, text):
    assert _read(driver, tmp_path, text, roundtrip=False) is None


def test_empty_entries(driver, tmp_path):
    assert _read(driver, tmp_path, '{"version": 1, "entries": {}}') == {}
